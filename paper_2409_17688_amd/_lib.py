"""ctypes binding of libtropical.so (the C ABI declared in include/tropical.h).

Each function here has the name of the C entry point it calls and does
argument marshalling only: it checks tensor dtypes, devices and strides,
passes raw device pointers, leading dimensions and the current HIP stream, and
turns a negative status into ``TropicalError``.  Every step of the computation
runs in the library's HIP kernels; PyTorch provides device memory and streams.
There is no fallback: when the library is missing, importing this module
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtropical.so")

TP_U8 = 1
TP_U16 = 2
TP_OK = 0
TP_EINVAL = -1
TP_ENOMEM = -2
TP_EOVERFLOW = -3
TP_EHIP = -4
TP_EBUSY = -5
TP_ECANCELED = -6
TP_PARAM_WAIT_LIMIT_US = 1
TP_PARAM_GRID = 2
TP_PARAM_FUSED_CHAIN = 3
TP_PARAM_COMPACT_FROM = 4
TP_PARAM_CHAIN_GIANTS_FROM = 5
TP_PARAM_BABY_STEPS = 32
TP_STEP_AUTO = 0
TP_STEP_CSR = 1
TP_STEP_BLOCKED = 2
TP_STEP_BLOCKED_ENTRIES = 3
TP_WALK_AUTO = 0
TP_WALK_CHAIN = 1
TP_WALK_STEPS = 2
TP_WALK_GEMV = 3
TP_COMPACT_GROUPED = 0x100

INF = {TP_U8: 255, TP_U16: 65535}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")

lib = ctypes.CDLL(LIB_PATH)


class Recurrence(ctypes.Structure):
    """tp_recurrence_t: A^(r0 + a) = b (x) A^r0 (Algorithm 3) from n0 on
    (Algorithm 4), found among the K powers compared `window` back."""
    _fields_ = [("found", ctypes.c_int32), ("window_short", ctypes.c_int32),
                ("K", ctypes.c_int32), ("window", ctypes.c_int32),
                ("r0", ctypes.c_int64), ("a", ctypes.c_int64), ("b", ctypes.c_int64),
                ("n0", ctypes.c_int64)]

    def __repr__(self):
        return (f"Recurrence(found={self.found}, window_short={self.window_short}, K={self.K}, "
                f"window={self.window}, r0={self.r0}, a={self.a}, b={self.b}, n0={self.n0})")


_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_i = ctypes.c_int

_SIGS = {
    "tp_last_error": ([], ctypes.c_char_p),
    "tp_version": ([], _i),
    "tp_state_dim": ([_i], _i64),
    "tp_state_nnz": ([_i], _i64),
    "tp_words": ([_i, _p, _p], _i),
    "tp_build_state_matrix": ([_i, _i, _p, _i64, _p], _i),
    "tp_build_state_csr": ([_i, _p, _p, _p, _p], _i),
    "tp_minplus_gemm": ([_i, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i, _p], _i),
    "tp_gemm_config_count": ([], _i),
    "tp_minplus_gemm_config": ([_i, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i, _i, _p],
                               _i),
    "tp_minplus_gemm_ex": ([_i, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i, _i, _i,
                            _p], _i),
    "tp_minplus_gemm_ex_noalloc": ([_i, _i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _i, _i,
                                    _i, _p], _i),
    "tp_tune_gemm": ([_i, _i64, _i, _i], _i),
    "tp_gemm_choice": ([_i, _i64, _i64, _i64, ctypes.POINTER(_i), ctypes.POINTER(_i)], _i),
    "tp_tune_planner": ([_i, ctypes.c_double, ctypes.c_double], _i),
    "tp_tune_batch": ([_i, _i, _i], _i),
    "tp_minplus_gemv": ([_i, _i64, _i64, _p, _i64, _p, _p, _i, _p], _i),
    "tp_minplus_spmm": ([_i, _i64, _i64, _p, _p, _p, _p, _i64, _p, _i64, _i64, _p], _i),
    "tp_state_left_mul": ([_i, _i, _p, _i64, _p, _i64, _i64, _p], _i),
    "tp_tune_step": ([_i, _i], _i),
    "tp_trace_min": ([_i, _i64, _p, _i64, _p, _p], _i),
    "tp_trace_of_product": ([_i, _i64, _p, _i64, _p, _i64, _p, _p], _i),
    "tp_sparse_trace_of_product": ([_i, _i64, _p, _p, _p, _p, _i64, _p, _p], _i),
    "tp_tropical_power_trace": ([_i, _i64, ctypes.POINTER(ctypes.c_int32), _p], _i),
    "tp_release_cache": ([], _i),
    "tp_apsp": ([_i, _i64, _p, _i64, _p, _i64, _p, _i64, _p], _i),
    "tp_state_select": ([_i, _i, _p, _i64, _p], _i64),
    "tp_build_state_columns": ([_i, _p, _i64, _p, _i64, _p], _i),
    "tp_diag_select_min": ([_i64, _i64, _p, _p, _i64, _p, _p], _i),
    "tp_tune_prune": ([_i], _i),
    "tp_compact_from_u16": ([_i64, _i64, _p, _i64, _p, _i64, _p, _p, _p], _i),
    "tp_compact_to_u16": ([_i64, _i64, _p, _i64, _p, _p, _i64, _p], _i),
    "tp_compact_step": ([_i, _p, _i64, _p, _p, _i64, _p, _i64, _p, _p], _i),
    "tp_compact_diag_min": ([_i64, _p, _i64, _p, _p, _p], _i),
    "tp_tune_compact_step": ([_i], _i),
    "tp_tune_compact_chains": ([_i], _i),
    "tp_compact_shared_from_u16": ([_i64, _i64, _p, _i64, _p, _i64, _p, _p, _p], _i),
    "tp_compact_shared_to_u16": ([_i64, _i64, _p, _i64, _p, _p, _i64, _p], _i),
    "tp_compact_shared_step": ([_i, _p, _i64, _p, _p, _i64, _p, _i64, _p, _p], _i),
    "tp_compact_shared_diag_min": ([_i64, _p, _i64, _p, _p, _p], _i),
    "tp_compact_shared_select_trace": ([_i64, _i64, _p, _p, _i64, _p, _p, _i64, _p, _p, _p],
                                       _i),
    "tp_const_diff": ([_i64, _p, _i64, _p, _i64, _p, _p], _i),
    "tp_recurrence": ([_i, _i, _i, ctypes.POINTER(Recurrence), ctypes.POINTER(ctypes.c_int32),
                       _p], _i),
    "tp_gamma2_recurrence": ([ctypes.POINTER(Recurrence), ctypes.POINTER(ctypes.c_int32), _i64,
                              ctypes.POINTER(_i64)], _i),
    "tp_ctx_create": ([ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)], _i),
    "tp_ctx_destroy": ([_p], _i),
    "tp_ctx_set_param": ([_p, _i, _i64], _i),
    "tp_ctx_resident_bytes": ([_p], _i64),
    "tp_ctx_need_bytes": ([_p, _i, _p, _p], _i64),
    "tp_ctx_release": ([_p, _i, _p], _i),
    "tp_ctx_copy_power": ([_p, _i, _i, _p, _i64, _p], _i),
    "tp_batch_power_trace": ([_p, _i, _p, _p, _p, _p], _i),
    "tp_ctx_check": ([_p, _p], _i),
    "tp_ctx_last_work": ([_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                         _i),
    "tp_cyclic_dim": ([_i], _i64),
    "tp_cyclic_nnz": ([_i], _i64),
    "tp_cyclic_words": ([_i, _p, _p], _i),
    "tp_build_cyclic_matrix": ([_i, _i, _p, _i64, _p], _i),
    "tp_build_cyclic_boundary": ([_i, _i, _p, _p, _p], _i),
    "tp_cyclic_walk_gamma2": ([_i64, _i, ctypes.POINTER(ctypes.c_int32), _p], _i),
    "tp_cyclic_walk_sweep": ([_i, _i64, _p, _i, _p], _i),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class TropicalError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what} (status {status})")
        self.status = status


def _check(rc: int) -> int:
    if rc < 0:
        raise TropicalError(rc, lib.tp_last_error().decode(errors="replace"))
    return rc


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint16:
        return TP_U16
    if t.dtype == torch.uint8:
        return TP_U8
    raise TypeError(f"expected a uint8 or uint16 tensor, got {t.dtype}")


def _torch_dtype(code: int):
    return torch.uint16 if code == TP_U16 else torch.uint8


def _mat(t: torch.Tensor, name: str):
    """(pointer, rows, cols, leading dimension) of a row-major device matrix."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    rows, cols = t.shape
    if cols > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    ld = t.stride(0) if rows > 1 else max(cols, 1)
    return t.data_ptr(), rows, cols, max(ld, cols, 1)


def _vec(t: torch.Tensor, name: str):
    if t.dim() != 1 or not t.is_cuda:
        raise ValueError(f"{name} must be a 1-D device tensor")
    if t.numel() > 1 and t.stride(0) != 1:
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


# ----------------------------------------------------------------- state --

def tp_version() -> int:
    return int(lib.tp_version())


def tp_state_dim(n: int) -> int:
    return _check(int(lib.tp_state_dim(n)))


def tp_state_nnz(n: int) -> int:
    return _check(int(lib.tp_state_nnz(n)))


def tp_words(n: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    N = tp_state_dim(n)
    if out is None:
        out = torch.empty(N, dtype=torch.int32, device="cuda")
    if out.numel() < N or out.element_size() != 4:
        raise ValueError("out must hold N 32-bit entries")
    _check(lib.tp_words(n, _vec(out, "out"), _stream(stream)))
    return out


def tp_build_state_matrix(n: int, dtype: int = TP_U16, out: torch.Tensor | None = None,
                          stream=None) -> torch.Tensor:
    N = tp_state_dim(n)
    if out is None:
        out = torch.empty((N, N), dtype=_torch_dtype(dtype), device="cuda")
    ptr, r, c, ld = _mat(out, "out")
    if r < N or c < N or _dtype_code(out) != dtype:
        raise ValueError("out must be at least N x N of the requested dtype")
    _check(lib.tp_build_state_matrix(n, dtype, ptr, ld, _stream(stream)))
    return out


def tp_build_state_csr(n: int, stream=None):
    """(rowptr int64[N+1], col int32[nnz] holding uint32 indices, z uint8[N])."""
    N = tp_state_dim(n)
    nnz = tp_state_nnz(n)
    rowptr = torch.empty(N + 1, dtype=torch.int64, device="cuda")
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    z = torch.empty(N, dtype=torch.uint8, device="cuda")
    _check(lib.tp_build_state_csr(n, rowptr.data_ptr(), col.data_ptr(), z.data_ptr(),
                                  _stream(stream)))
    return rowptr, col[:nnz], z


# -------------------------------------------------------------- products --

def tp_gemm_config_count() -> int:
    return int(lib.tp_gemm_config_count())


def tp_minplus_gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
                    accumulate: bool = False, config: int | None = None,
                    ksplit: int | None = None, stream=None) -> torch.Tensor:
    """C = A x B (min with the old C when accumulate).  config=None uses the
    library's default (tuned) shape; config with ksplit calls
    tp_minplus_gemm_ex, config alone tp_minplus_gemm_config."""
    dt = _dtype_code(A)
    if _dtype_code(B) != dt:
        raise TypeError("A and B must have the same dtype")
    pa, M, K, lda = _mat(A, "A")
    pb, K2, N, ldb = _mat(B, "B")
    if K2 != K:
        raise ValueError(f"inner dimensions differ: {K} vs {K2}")
    if C is None:
        if accumulate:
            raise ValueError("accumulate needs C")
        C = torch.empty((M, N), dtype=A.dtype, device=A.device)
    pc, M2, N2, ldc = _mat(C, "C")
    if (M2, N2) != (M, N) or _dtype_code(C) != dt:
        raise ValueError("C has the wrong shape or dtype")
    if config is None:
        if ksplit is not None:
            raise ValueError("ksplit needs an explicit config")
        _check(lib.tp_minplus_gemm(dt, M, N, K, pa, lda, pb, ldb, pc, ldc, int(accumulate),
                                   _stream(stream)))
    elif ksplit is not None:
        _check(lib.tp_minplus_gemm_ex(dt, M, N, K, pa, lda, pb, ldb, pc, ldc, int(accumulate),
                                      int(config), int(ksplit), _stream(stream)))
    else:
        _check(lib.tp_minplus_gemm_config(dt, M, N, K, pa, lda, pb, ldb, pc, ldc,
                                          int(accumulate), int(config), _stream(stream)))
    return C


def tp_minplus_gemm_ex(A, B, C=None, accumulate=False, config=0, ksplit=1, stream=None):
    return tp_minplus_gemm(A, B, C, accumulate, config=config, ksplit=ksplit, stream=stream)


# ---------------------------------------------------------------- tuning --

def tp_tune_gemm(dtype: int, max_dim: int, config: int = 0, ksplit: int = 1) -> None:
    _check(lib.tp_tune_gemm(int(dtype), int(max_dim), int(config), int(ksplit)))


def tp_gemm_choice(dtype: int, M: int, N: int, K: int) -> tuple[int, int]:
    cfg, ks = ctypes.c_int(-1), ctypes.c_int(-1)
    _check(lib.tp_gemm_choice(int(dtype), int(M), int(N), int(K), ctypes.byref(cfg),
                              ctypes.byref(ks)))
    return int(cfg.value), int(ks.value)


def tp_tune_planner(n: int, spmm_ops_per_s: float, gemm_ops_per_s: float) -> None:
    _check(lib.tp_tune_planner(int(n), float(spmm_ops_per_s), float(gemm_ops_per_s)))


def tp_tune_batch(n: int, baby_steps: int, fused_baby_steps: int = 0) -> None:
    _check(lib.tp_tune_batch(int(n), int(baby_steps), int(fused_baby_steps)))


def tp_minplus_gemv(A: torch.Tensor, x: torch.Tensor, trans: bool = False,
                    y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    dt = _dtype_code(A)
    if _dtype_code(x) != dt:
        raise TypeError("A and x must have the same dtype")
    pa, M, K, lda = _mat(A, "A")
    nx, ny = (M, K) if trans else (K, M)
    if x.numel() != nx:
        raise ValueError(f"x must have {nx} entries")
    if y is None:
        y = torch.empty(ny, dtype=A.dtype, device=A.device)
    if y.numel() != ny or _dtype_code(y) != dt:
        raise ValueError("y has the wrong size or dtype")
    _check(lib.tp_minplus_gemv(dt, M, K, pa, lda, _vec(x, "x") if nx else None,
                               _vec(y, "y") if ny else None, int(trans), _stream(stream)))
    return y


def tp_minplus_spmm(rowptr: torch.Tensor, col: torch.Tensor, z: torch.Tensor, X: torch.Tensor,
                    Y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    dt = _dtype_code(X)
    rows = rowptr.numel() - 1
    px, K, ncols, ldx = _mat(X, "X")
    if Y is None:
        Y = torch.empty((rows, ncols), dtype=X.dtype, device=X.device)
    py, r2, c2, ldy = _mat(Y, "Y")
    if (r2, c2) != (rows, ncols) or _dtype_code(Y) != dt:
        raise ValueError("Y has the wrong shape or dtype")
    if rowptr.dtype != torch.int64 or col.element_size() != 4 or z.dtype != torch.uint8:
        raise TypeError("rowptr int64, col 32-bit, z uint8")
    _check(lib.tp_minplus_spmm(dt, rows, K, _vec(rowptr, "rowptr"),
                               col.data_ptr() if col.numel() else None, _vec(z, "z"), px, ldx,
                               py, ldy, ncols, _stream(stream)))
    return Y


def tp_state_left_mul(n: int, X: torch.Tensor, Y: torch.Tensor | None = None,
                      form: int = 0, stream=None) -> torch.Tensor:
    """Y = A(D_n) x X for a u16 X with N = tp_state_dim(n) rows; form is
    TP_STEP_AUTO, TP_STEP_CSR or TP_STEP_BLOCKED."""
    if X.dtype != torch.uint16:
        raise TypeError("X must be uint16")
    N = tp_state_dim(n)
    px, rows, ncols, ldx = _mat(X, "X")
    if rows != N:
        raise ValueError(f"X must have {N} rows")
    if Y is None:
        Y = torch.empty((N, ncols), dtype=X.dtype, device=X.device)
    py, r2, c2, ldy = _mat(Y, "Y")
    if (r2, c2) != (N, ncols) or Y.dtype != torch.uint16:
        raise ValueError("Y has the wrong shape or dtype")
    _check(lib.tp_state_left_mul(int(n), int(form), px, ldx, py, ldy, ncols, _stream(stream)))
    return Y


def tp_tune_step(n: int, form: int) -> None:
    _check(lib.tp_tune_step(int(n), int(form)))


# ---------------------------------------------------------------- traces --

def _scalar_out(out):
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device="cuda")
    return out


def tp_trace_min(X: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    dt = _dtype_code(X)
    px, N, N2, ldx = _mat(X, "X")
    if N != N2:
        raise ValueError("X must be square")
    out = _scalar_out(out)
    _check(lib.tp_trace_min(dt, N, px, ldx, out.data_ptr(), _stream(stream)))
    return out


def tp_trace_of_product(X: torch.Tensor, Y: torch.Tensor, out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    dt = _dtype_code(X)
    if _dtype_code(Y) != dt:
        raise TypeError("X and Y must have the same dtype")
    px, N, N2, ldx = _mat(X, "X")
    py, N3, N4, ldy = _mat(Y, "Y")
    if not (N == N2 == N3 == N4):
        raise ValueError("X and Y must be square of one size")
    out = _scalar_out(out)
    _check(lib.tp_trace_of_product(dt, N, px, ldx, py, ldy, out.data_ptr(), _stream(stream)))
    return out


def tp_sparse_trace_of_product(rowptr, col, z, X: torch.Tensor, out=None, stream=None):
    dt = _dtype_code(X)
    px, N, N2, ldx = _mat(X, "X")
    if N != N2 or rowptr.numel() != N + 1:
        raise ValueError("X must be N x N with rowptr of N + 1 entries")
    out = _scalar_out(out)
    _check(lib.tp_sparse_trace_of_product(dt, N, _vec(rowptr, "rowptr"),
                                          col.data_ptr() if col.numel() else None, _vec(z, "z"),
                                          px, ldx, out.data_ptr(), _stream(stream)))
    return out


# --------------------------------------------------------------- gamma_2 --

def tp_tropical_power_trace(n: int, m: int, stream=None) -> int:
    """gamma_2(P_n x C_m) = min_i (A(D_n)^m)_ii (Theorem 2); blocks."""
    res = ctypes.c_int32(-1)
    _check(lib.tp_tropical_power_trace(n, m, ctypes.byref(res), _stream(stream)))
    return int(res.value)


def tp_const_diff(X: torch.Tensor, Y: torch.Tensor, out: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """out (device int32[2]) = {min, max} of the finite entries of X - Y, see
    the C declaration for the INF cases."""
    if X.dtype != torch.uint16 or Y.dtype != torch.uint16:
        raise TypeError("X and Y must be uint16")
    px, N, N2, ldx = _mat(X, "X")
    py, N3, N4, ldy = _mat(Y, "Y")
    if not (N == N2 == N3 == N4):
        raise ValueError("X and Y must be square of one size")
    # the row stride as allocated, also for one row (the kernel reads rows in
    # 16-byte chunks of one common leading dimension)
    ldx, ldy = max(X.stride(0), N), max(Y.stride(0), N)
    if out is None:
        out = torch.empty(2, dtype=torch.int32, device=X.device)
    _check(lib.tp_const_diff(N, px, ldx, py, ldy, out.data_ptr(), _stream(stream)))
    return out


def tp_recurrence(n: int, K: int = 50, window: int = 0, stream=None):
    """(Recurrence, diag_min) for A(D_n)^1 .. A(D_n)^K; diag_min[k - 1] =
    min_i (A^k)_ii, a host int32 array.  Blocks until done."""
    import numpy as np
    rec = Recurrence()
    diag = np.zeros(max(int(K), 1), dtype=np.int32)
    _check(lib.tp_recurrence(int(n), int(K), int(window), ctypes.byref(rec),
                             diag.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             _stream(stream)))
    return rec, diag


def tp_gamma2_recurrence(rec: Recurrence, diag_min, m: int) -> int:
    """gamma_2(P_n x C_m) for any m >= 3 from tp_recurrence's results (host)."""
    import numpy as np
    diag = np.ascontiguousarray(diag_min, dtype=np.int32)
    if diag.ndim != 1 or diag.shape[0] < rec.K:
        raise ValueError(f"diag_min must hold the {rec.K} diagonal minima")
    out = ctypes.c_int64(0)
    _check(lib.tp_gamma2_recurrence(ctypes.byref(rec),
                                    diag.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    int(m), ctypes.byref(out)))
    return int(out.value)


def tp_state_select(n: int, max_zeros: int, stream=None) -> torch.Tensor:
    """Device int32 indices of the states of A(D_n) with at most max_zeros zeros."""
    cnt = _check(lib.tp_state_select(int(n), int(max_zeros), None, 0, _stream(stream)))
    out = torch.empty(max(cnt, 1), dtype=torch.int32, device="cuda")
    _check(lib.tp_state_select(int(n), int(max_zeros), out.data_ptr(), out.numel(),
                               _stream(stream)))
    return out[:cnt]


def tp_build_state_columns(n: int, idx: torch.Tensor, out: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    """Columns idx of A(D_n) (u16, N x len(idx))."""
    if idx.dtype != torch.int32 or not idx.is_cuda or idx.dim() != 1:
        raise TypeError("idx must be a 1-D device int32 tensor")
    idx = idx.contiguous()
    N, cnt = tp_state_dim(n), idx.numel()
    if out is None:
        ld = max((cnt + 63) // 64 * 64, 64)
        out = torch.empty((N, ld), dtype=torch.uint16, device="cuda")[:, :cnt]
    px, rows, cols, ldx = _mat(out, "out")
    if (rows, cols) != (N, cnt) or out.dtype != torch.uint16:
        raise ValueError(f"out must be a ({N}, {cnt}) uint16 matrix")
    _check(lib.tp_build_state_columns(int(n), idx.data_ptr(), cnt, px, max(out.stride(0), cnt),
                                      _stream(stream)))
    return out


def tp_diag_select_min(X: torch.Tensor, idx: torch.Tensor, out: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """out (device int32[1]) = min_j X[idx[j], j]."""
    if X.dtype != torch.uint16:
        raise TypeError("X must be uint16")
    if idx.dtype != torch.int32 or not idx.is_cuda or idx.dim() != 1:
        raise TypeError("idx must be a 1-D device int32 tensor")
    idx = idx.contiguous()
    px, rows, cols, ldx = _mat(X, "X")
    if cols < idx.numel():
        raise ValueError("X has fewer columns than idx has entries")
    out = _scalar_out(out)
    _check(lib.tp_diag_select_min(rows, idx.numel(), idx.data_ptr(), px,
                                  max(X.stride(0) if rows else 0, idx.numel()), out.data_ptr(),
                                  _stream(stream)))
    return out


def tp_tune_prune(mode: int) -> None:
    _check(lib.tp_tune_prune(int(mode)))


def tp_apsp(W: torch.Tensor, D: torch.Tensor | None = None, T: torch.Tensor | None = None,
            stream=None) -> torch.Tensor:
    """All-pairs shortest paths: D = min(distance, INF) for the arc weights W
    (INF = no arc), by (min,+) squaring."""
    dt = _dtype_code(W)
    pw, N, N2, ldw = _mat(W, "W")
    if N != N2:
        raise ValueError("W must be square")
    if D is None:
        D = torch.empty_like(W)
    if T is None:
        T = torch.empty_like(W)
    for name, M in (("D", D), ("T", T)):
        if M.dtype != W.dtype or tuple(M.shape) != (N, N):
            raise ValueError(f"{name} must match W")
    pd, _, _, ldd = _mat(D, "D")
    pt, _, _, ldt = _mat(T, "T")
    _check(lib.tp_apsp(dt, N, pw, ldw, pd, ldd, pt, ldt, _stream(stream)))
    return D


# ---------------------------------------------------------- compact powers --
COMPACT_DEAD = 0x3FFFFFFF
COMPACT_RANGE, COMPACT_MIXED = 1, 2


def _u8rows(M: torch.Tensor, name: str, ncols: int):
    if M.dtype != torch.uint8 or M.dim() != 2 or M.device.type != "cuda":
        raise ValueError(f"{name} must be a 2-D uint8 CUDA tensor")
    if M.stride(1) != 1 or M.shape[1] < ncols:
        raise ValueError(f"{name} needs unit column stride and at least {ncols} columns")
    return ctypes.c_void_p(M.data_ptr()), M.shape[0], M.stride(0)


def tp_compact_from_u16(X: torch.Tensor, Y: torch.Tensor | None = None,
                        R: torch.Tensor | None = None, status: torch.Tensor | None = None,
                        stream=None):
    """(Y, R): the compact form of the 16-bit matrix X (u8 residuals, one
    int32 offset per row).  Bits of ``status`` (int32 CUDA tensor of one
    element, ORed into): COMPACT_RANGE, COMPACT_MIXED."""
    if X.dtype != torch.uint16:
        raise ValueError("X must be uint16")
    px, N, ncols, ldx = _mat(X, "X")
    if Y is None:
        Y = torch.empty((N, (ncols + 7) // 8 * 8 or 8), dtype=torch.uint8, device=X.device)
    if R is None:
        R = torch.empty(max(N, 1), dtype=torch.int32, device=X.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    py, Ny, ldy = _u8rows(Y, "Y", ncols)
    if Ny != N or R.numel() < N or R.dtype != torch.int32:
        raise ValueError("Y must have N rows and R N int32 entries")
    _check(lib.tp_compact_from_u16(N, ncols, px, ldx, py, ldy, ctypes.c_void_p(R.data_ptr()),
                                   ctypes.c_void_p(status.data_ptr()), _stream(stream)))
    return Y, R


def tp_compact_to_u16(X: torch.Tensor, R: torch.Tensor, ncols: int,
                      Y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The 16-bit form (N x ncols) of the compact matrix (X, R)."""
    px, N, ldx = _u8rows(X, "X", ncols)
    if Y is None:
        Y = torch.empty((N, ncols), dtype=torch.uint16, device=X.device)
    py, Ny, nc, ldy = _mat(Y, "Y")
    if Ny != N or nc != ncols or R.numel() < N or R.dtype != torch.int32:
        raise ValueError("Y must be N x ncols and R N int32 entries")
    _check(lib.tp_compact_to_u16(N, ncols, px, ldx, ctypes.c_void_p(R.data_ptr()), py, ldy,
                                 _stream(stream)))
    return Y


def tp_compact_step(n: int, X: torch.Tensor, RX: torch.Tensor, ncols: int,
                    Y: torch.Tensor | None = None, RY: torch.Tensor | None = None,
                    status: torch.Tensor | None = None, stream=None):
    """(Y, RY) = A(D_n) x (X, RX) in compact form."""
    px, N, ldx = _u8rows(X, "X", ncols)
    if Y is None:
        Y = torch.empty_like(X)
    if RY is None:
        RY = torch.empty_like(RX)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    py, Ny, ldy = _u8rows(Y, "Y", ncols)
    if Ny != N or RX.dtype != torch.int32 or RY.dtype != torch.int32 or \
            RX.numel() < N or RY.numel() < N:
        raise ValueError("Y must have N rows and RX, RY N int32 entries")
    _check(lib.tp_compact_step(int(n), px, ldx, ctypes.c_void_p(RX.data_ptr()), py, ldy,
                               ctypes.c_void_p(RY.data_ptr()), int(ncols),
                               ctypes.c_void_p(status.data_ptr()), _stream(stream)))
    return Y, RY


def tp_compact_diag_min(X: torch.Tensor, R: torch.Tensor, stream=None) -> int:
    """Diagonal minimum of a square compact power (Theorem 2)."""
    px, N, ldx = _u8rows(X, "X", X.shape[0])
    out = torch.empty(1, dtype=torch.int32, device=X.device)
    _check(lib.tp_compact_diag_min(N, px, ldx, ctypes.c_void_p(R.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return int(out.item())


def _base(t, name):
    if t.dtype != torch.int32 or t.numel() < 2 or not t.is_cuda:
        raise ValueError(f"{name} must be an int32 CUDA tensor of two elements")
    return ctypes.c_void_p(t.data_ptr())


def tp_compact_shared_from_u16(X: torch.Tensor, Y: torch.Tensor | None = None,
                               base: torch.Tensor | None = None,
                               status: torch.Tensor | None = None, stream=None):
    """(Y, base): the shared-base compact form of the 16-bit matrix X
    (base = [G, least residual])."""
    if X.dtype != torch.uint16:
        raise ValueError("X must be uint16")
    px, N, ncols, ldx = _mat(X, "X")
    if Y is None:
        Y = torch.empty((N, (ncols + 7) // 8 * 8 or 8), dtype=torch.uint8, device=X.device)
    if base is None:
        base = torch.empty(2, dtype=torch.int32, device=X.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    py, Ny, ldy = _u8rows(Y, "Y", ncols)
    if Ny != N:
        raise ValueError("Y must have N rows")
    _check(lib.tp_compact_shared_from_u16(N, ncols, px, ldx, py, ldy, _base(base, "base"),
                                          ctypes.c_void_p(status.data_ptr()), _stream(stream)))
    return Y, base


def tp_compact_shared_to_u16(X: torch.Tensor, base: torch.Tensor, ncols: int,
                             Y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    px, N, ldx = _u8rows(X, "X", ncols)
    if Y is None:
        Y = torch.empty((N, ncols), dtype=torch.uint16, device=X.device)
    py, Ny, nc, ldy = _mat(Y, "Y")
    if Ny != N or nc != ncols:
        raise ValueError("Y must be N x ncols")
    _check(lib.tp_compact_shared_to_u16(N, ncols, px, ldx, _base(base, "base"), py, ldy,
                                        _stream(stream)))
    return Y


def tp_compact_shared_step(n: int, X: torch.Tensor, bx: torch.Tensor, ncols: int,
                           Y: torch.Tensor | None = None, by: torch.Tensor | None = None,
                           status: torch.Tensor | None = None, stream=None):
    """(Y, by) = A(D_n) x (X, bx) in shared-base compact form."""
    px, N, ldx = _u8rows(X, "X", ncols)
    if Y is None:
        Y = torch.empty_like(X)
    if by is None:
        by = torch.empty_like(bx)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
    py, Ny, ldy = _u8rows(Y, "Y", ncols)
    if Ny != N:
        raise ValueError("Y must have N rows")
    _check(lib.tp_compact_shared_step(int(n), px, ldx, _base(bx, "bx"), py, ldy, _base(by, "by"),
                                      int(ncols), ctypes.c_void_p(status.data_ptr()),
                                      _stream(stream)))
    return Y, by


def tp_compact_shared_diag_min(X: torch.Tensor, base: torch.Tensor, stream=None) -> int:
    px, N, ldx = _u8rows(X, "X", X.shape[0])
    out = torch.empty(1, dtype=torch.int32, device=X.device)
    _check(lib.tp_compact_shared_diag_min(N, px, ldx, _base(base, "base"),
                                          ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return int(out.item())


def tp_compact_shared_select_trace(X: torch.Tensor, bx: torch.Tensor, P: torch.Tensor,
                                   bp: torch.Tensor, idx: torch.Tensor | None = None,
                                   out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """out[0] = G_X + G_P + min over t of min_k x[r_t][k] + p[k][t] (saturated
    at 65535): the trace of X x P on the diagonal entries of the states
    idx (all N states when idx is None; then P is N x N)."""
    px, N, ldx = _u8rows(X, "X", 0)
    if X.shape[1] < N:
        raise ValueError("X must be N x N")
    count = int(idx.numel()) if idx is not None else N
    pp, Np, ldp = _u8rows(P, "P", count)
    if Np != N or P.shape[1] < count:
        raise ValueError("P must be N x count")
    if idx is not None and idx.dtype != torch.int32:
        raise TypeError("idx must be int32")
    out = _scalar_out(out)
    _check(lib.tp_compact_shared_select_trace(
        N, count, ctypes.c_void_p(idx.data_ptr()) if idx is not None else None, px, ldx,
        _base(bx, "bx"), pp, ldp, _base(bp, "bp"), ctypes.c_void_p(out.data_ptr()),
        _stream(stream)))
    return out


def tp_tune_compact_chains(compact_from_n: int) -> None:
    """Path orders from which the recurrence and the pruned plain path chain
    compact powers (0: never)."""
    _check(lib.tp_tune_compact_chains(int(compact_from_n)))


def tp_tune_compact_step(unroll: int) -> None:
    _check(lib.tp_tune_compact_step(int(unroll)))


def tp_release_cache() -> None:
    _check(lib.tp_release_cache())


def tp_last_error() -> str:
    return lib.tp_last_error().decode(errors="replace")


# --------------------------------------------------------------- batching --

def tp_ctx_create(hbm_budget_bytes: int) -> int:
    h = ctypes.c_void_p()
    _check(lib.tp_ctx_create(int(hbm_budget_bytes), ctypes.byref(h)))
    return h.value


def tp_ctx_destroy(ctx: int) -> None:
    _check(lib.tp_ctx_destroy(ctx))


def tp_ctx_set_param(ctx: int, param: int, value: int) -> None:
    _check(lib.tp_ctx_set_param(ctx, int(param), int(value)))


def tp_ctx_resident_bytes(ctx: int) -> int:
    return _check(int(lib.tp_ctx_resident_bytes(ctx)))


def tp_ctx_release(ctx: int, n: int = 0, stream=None) -> None:
    _check(lib.tp_ctx_release(ctx, int(n), _stream(stream)))


def tp_ctx_copy_power(ctx: int, n: int, e: int, out: torch.Tensor | None = None,
                      stream=None) -> torch.Tensor:
    """The context's resident power A(D_n)^e as a device uint16 tensor of
    shape (N, N) (or into `out`, rows of stride >= N)."""
    N = tp_state_dim(n)
    if out is None:
        out = torch.empty((N, N), dtype=torch.uint16, device="cuda")
    po, rows, ncols, ld = _mat(out, "out")
    if (rows, ncols) != (N, N) or out.dtype != torch.uint16:
        raise ValueError(f"out must be uint16 of shape ({N}, {N})")
    _check(lib.tp_ctx_copy_power(ctx, int(n), int(e), po, ld, _stream(stream)))
    return out


def tp_ctx_need_bytes(ctx: int, ns, ms) -> int:
    import numpy as np
    n_arr = np.ascontiguousarray(ns, dtype=np.int32)
    m_arr = np.ascontiguousarray(ms, dtype=np.int64)
    return _check(int(lib.tp_ctx_need_bytes(ctx, int(n_arr.size), n_arr.ctypes.data,
                                            m_arr.ctypes.data)))


def tp_batch_power_trace(ctx: int, ns, ms, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
    """Queues gamma_2 for every (ns[j], ms[j]); returns the device int32 result
    tensor (valid once tp_ctx_check has returned)."""
    import numpy as np
    n_arr = np.ascontiguousarray(ns, dtype=np.int32)
    m_arr = np.ascontiguousarray(ms, dtype=np.int64)
    if n_arr.shape != m_arr.shape or n_arr.ndim != 1:
        raise ValueError("ns and ms must be 1-D of one length")
    count = int(n_arr.size)
    if out is None:
        out = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    if out.numel() < count or out.dtype != torch.int32:
        raise ValueError("out must hold count int32 entries")
    _check(lib.tp_batch_power_trace(ctx, count, n_arr.ctypes.data, m_arr.ctypes.data,
                                    out.data_ptr(), _stream(stream)))
    return out[:count]


def tp_ctx_check(ctx: int, stream=None) -> None:
    _check(lib.tp_ctx_check(ctx, _stream(stream)))


# -- small cycle, any path: columns that are copies of C_m ------------------

def tp_cyclic_dim(m: int) -> int:
    """Number of correct cyclic words of length m (3 <= m <= 12)."""
    return _check(int(lib.tp_cyclic_dim(m)))


def tp_cyclic_nnz(m: int) -> int:
    return _check(int(lib.tp_cyclic_nnz(m)))


def tp_cyclic_words(m: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Base-3 codes of the correct cyclic words (int32 tensor holding uint32)."""
    N = tp_cyclic_dim(m)
    if out is None:
        out = torch.empty(N, dtype=torch.int32, device="cuda")
    if out.dtype != torch.int32 or out.numel() < N or not out.is_cuda:
        raise ValueError("out must be a cuda int32 tensor of at least N entries")
    _check(lib.tp_cyclic_words(m, out.data_ptr(), _stream(stream)))
    return out


def tp_build_cyclic_matrix(m: int, dtype: int = TP_U16, out: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    """The cyclic column digraph's N x N matrix in 8 or 16 bits."""
    N = tp_cyclic_dim(m)
    if out is None:
        out = torch.empty((N, N), dtype=_torch_dtype(dtype), device="cuda")
    ptr, r, c, ld = _mat(out, "out")
    if r < N or c < N or _dtype_code(out) != dtype:
        raise ValueError("out must be at least N x N of the requested dtype")
    _check(lib.tp_build_cyclic_matrix(m, dtype, ptr, ld, _stream(stream)))
    return out


def tp_build_cyclic_boundary(m: int, dtype: int = TP_U16, stream=None):
    """(start, end) vectors of the walk along the path, N entries each."""
    N = tp_cyclic_dim(m)
    start = torch.empty(N, dtype=_torch_dtype(dtype), device="cuda")
    end = torch.empty(N, dtype=_torch_dtype(dtype), device="cuda")
    _check(lib.tp_build_cyclic_boundary(m, dtype, start.data_ptr(), end.data_ptr(),
                                        _stream(stream)))
    return start, end


def tp_cyclic_walk_gamma2(n: int, m: int, stream=None) -> int:
    """gamma_2(P_n x C_m) by n - 1 dense vector-matrix products over cyclic
    columns; blocks."""
    res = ctypes.c_int32(-1)
    _check(lib.tp_cyclic_walk_gamma2(n, m, ctypes.byref(res), _stream(stream)))
    return int(res.value)


def tp_cyclic_walk_sweep(m: int, nmax: int, out: torch.Tensor | None = None,
                         form: int = TP_WALK_AUTO, stream=None) -> torch.Tensor:
    """out[k - 1] (device int32) = gamma_2(P_k x C_m) for k = 1..nmax."""
    if out is None:
        out = torch.empty(max(nmax, 1), dtype=torch.int32, device="cuda")
    if out.dtype != torch.int32 or out.numel() < nmax or not out.is_cuda:
        raise ValueError("out must be a cuda int32 tensor of at least nmax entries")
    _check(lib.tp_cyclic_walk_sweep(m, nmax, out.data_ptr(), form, _stream(stream)))
    return out


def tp_ctx_last_work(ctx) -> dict:
    """Algorithmic work of the last batch queued on ctx: (min,+) operations of
    its chain levels, dense products and traces, and their least bytes."""
    ops = (ctypes.c_double * 3)()
    nbytes = ctypes.c_double(0)
    _check(lib.tp_ctx_last_work(ctx, ops, ctypes.byref(nbytes)))
    return {"chain_ops": ops[0], "product_ops": ops[1], "trace_ops": ops[2],
            "ops": ops[0] + ops[1] + ops[2], "bytes": nbytes.value}
