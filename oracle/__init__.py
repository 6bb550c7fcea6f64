"""CPU oracle for the 2-domination number of cylinders by (min,+) powers.

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product library
never does.  It shares no code with the HIP path.

The arithmetic lives in two plain C files compiled with gcc:

* ``oracle.c``   -- correct words and arcs (Section 2.2), the state matrix
  (Algorithm 1), the (min,+) product (Section 1), the power chain
  (Algorithm 2), gamma_2 as the diagonal minimum (Theorem 2, Algorithm 5),
  the recurrence search (Algorithms 3 and 4) and the complementary
  construction (columns that are copies of the cycle, an open walk along the
  path by (min,+) vector-matrix products: the small-cycle / any-path problem
  Section 1 names, on the general construction of Section 2.1);
* ``brute2dom.c`` -- exhaustive search for minimum 2-dominating sets straight
  from the definition (Section 1), used as an independent pin.

Every matrix crosses this interface as int32 with an explicit INF (65535 for
16-bit storage, 255 for 8-bit storage, Section 3 uses 16-bit integers);
callers convert to and from the storage type.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "brute2dom.c")]

INF16 = 65535
INF8 = 255

_lib = None


def build() -> str:
    """Compile the oracle's C sources into ``oracle/_oracle.so`` (always)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
           "-std=c11", "-Wall", "-Wextra", "-o", _SO + ".tmp"] + _SOURCES
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_is_correct_word.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_is_correct_word.restype = ctypes.c_int
    lib.oracle_words.argtypes = [ctypes.c_int, u32p]
    lib.oracle_words.restype = ctypes.c_int64
    lib.oracle_zeros.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_zeros.restype = ctypes.c_int
    lib.oracle_follows.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_follows.restype = ctypes.c_int
    lib.oracle_state_matrix.argtypes = [ctypes.c_int, ctypes.c_int32, i32p]
    lib.oracle_state_matrix.restype = ctypes.c_int64
    lib.oracle_state_rows.argtypes = [ctypes.c_int, ctypes.c_int64, i64p, ctypes.c_int32, i32p]
    lib.oracle_state_rows.restype = ctypes.c_int64
    lib.oracle_minplus.argtypes = [ctypes.c_int64] * 3 + [i32p, ctypes.c_int64, i32p, ctypes.c_int64,
                                                          i32p, ctypes.c_int64, ctypes.c_int32]
    lib.oracle_minplus.restype = None
    lib.oracle_trace_min.argtypes = [ctypes.c_int64, i32p, ctypes.c_int64, ctypes.c_int32]
    lib.oracle_trace_min.restype = ctypes.c_int32
    lib.oracle_gamma2_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int32, i32p]
    lib.oracle_gamma2_sweep.restype = ctypes.c_int64
    lib.oracle_power.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int32, i32p]
    lib.oracle_power.restype = ctypes.c_int64
    lib.oracle_recurrence.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int32, i64p]
    lib.oracle_recurrence.restype = ctypes.c_int
    lib.oracle_apsp.argtypes = [ctypes.c_int64, i32p, ctypes.c_int32, i32p]
    lib.oracle_apsp.restype = None
    lib.oracle_constant_difference.argtypes = [ctypes.c_int64, i32p, i32p, ctypes.c_int32, i64p]
    lib.oracle_constant_difference.restype = ctypes.c_int
    lib.oracle_is_correct_cyclic_word.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_is_correct_cyclic_word.restype = ctypes.c_int
    lib.oracle_cyclic_words.argtypes = [ctypes.c_int, u32p]
    lib.oracle_cyclic_words.restype = ctypes.c_int64
    lib.oracle_cyclic_follows.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_cyclic_follows.restype = ctypes.c_int
    lib.oracle_cyclic_can_start.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_cyclic_can_start.restype = ctypes.c_int
    lib.oracle_cyclic_can_end.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_cyclic_can_end.restype = ctypes.c_int
    lib.oracle_cyclic_state_matrix.argtypes = [ctypes.c_int, ctypes.c_int32, i32p]
    lib.oracle_cyclic_state_matrix.restype = ctypes.c_int64
    lib.oracle_cyclic_boundary.argtypes = [ctypes.c_int, ctypes.c_int32, i32p, i32p]
    lib.oracle_cyclic_boundary.restype = ctypes.c_int64
    lib.oracle_path_gamma2_sweep.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int32, i32p]
    lib.oracle_path_gamma2_sweep.restype = ctypes.c_int64
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.brute_is_2dominating.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64]
    lib.brute_is_2dominating.restype = ctypes.c_int
    lib.brute_gamma2.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.brute_gamma2.restype = ctypes.c_int
    _lib = lib
    return lib


def _i32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def word_count(n: int) -> int:
    """|C_n|, the number of correct words of length n (Section 2.2, Table 1)."""
    return int(_load().oracle_words(n, None))


def words(n: int) -> np.ndarray:
    """Base-3 codes of the correct words, increasing (p^1 most significant)."""
    N = word_count(n)
    out = np.zeros(N, dtype=np.uint32)
    _load().oracle_words(n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def word_string(n: int, code: int) -> str:
    digits = []
    for _ in range(n):
        digits.append(str(code % 3))
        code //= 3
    return "".join(reversed(digits))


def is_correct_word(n: int, code: int) -> bool:
    return bool(_load().oracle_is_correct_word(n, code))


def follows(n: int, q: int, p: int) -> bool:
    """True when word p can follow word q (Section 2.2)."""
    return bool(_load().oracle_follows(n, q, p))


def zeros(n: int, code: int) -> int:
    return int(_load().oracle_zeros(n, code))


def state_matrix(n: int, inf: int = INF16) -> np.ndarray:
    """A(D_n) as an N x N int32 matrix (Algorithm 1)."""
    N = word_count(n)
    A = np.empty((N, N), dtype=np.int32)
    _load().oracle_state_matrix(n, inf, _i32(A))
    return A


def state_rows(n: int, rows, inf: int = INF16) -> np.ndarray:
    """Rows ``rows`` of A(D_n) (Algorithm 1) as a len(rows) x N int32 matrix,
    without building the whole matrix (n = 11, 12)."""
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    N = word_count(n)
    out = np.empty((rows.size, N), dtype=np.int32)
    r = _load().oracle_state_rows(n, rows.size, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  inf, _i32(out))
    if r < 0:
        raise ValueError("bad path order or row index")
    return out


def minplus(A: np.ndarray, B: np.ndarray, inf: int = INF16) -> np.ndarray:
    """(min,+) product of two matrices with entries in [0, inf], saturating."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.empty((M, N), dtype=np.int32)
    _load().oracle_minplus(M, N, K, _i32(A), K, _i32(B), N, _i32(C), N, inf)
    return C


def minplus_rows(A: np.ndarray, B: np.ndarray, rows, inf: int = INF16) -> np.ndarray:
    """Selected rows of A x B: each is (row of A) x B by the same product."""
    rows = np.asarray(rows, dtype=np.int64)
    return minplus(np.asarray(A)[rows], B, inf)


def trace_min(X: np.ndarray, inf: int = INF16) -> int:
    X = np.ascontiguousarray(X, dtype=np.int32)
    N = X.shape[0]
    return int(_load().oracle_trace_min(N, _i32(X), X.shape[1], inf))


def power(n: int, k: int, inf: int = INF16) -> np.ndarray:
    """A(D_n)^k by Algorithm 2."""
    N = word_count(n)
    X = np.empty((N, N), dtype=np.int32)
    _load().oracle_power(n, k, inf, _i32(X))
    return X


def gamma2_sweep(n: int, kmax: int, inf: int = INF16) -> np.ndarray:
    """g[k-1] = min_i (A^k)_ii for k = 1..kmax; g[m-1] = gamma_2(P_n x C_m) for m >= 3."""
    g = np.empty(kmax, dtype=np.int32)
    _load().oracle_gamma2_sweep(n, kmax, inf, _i32(g))
    return g


def gamma2(n: int, m: int, inf: int = INF16) -> int:
    """gamma_2(P_n x C_m) = min_i (A(D_n)^m)_ii (Theorem 2), m >= 3."""
    if m < 3:
        raise ValueError("the cycle order m must be at least 3")
    return int(gamma2_sweep(n, m, inf)[m - 1])


def recurrence(n: int, K: int = 50, inf: int = INF16):
    """(r0, a, b, m0) from Algorithms 3 and 4 on the first K powers, or None."""
    out = np.zeros(4, dtype=np.int64)
    ok = _load().oracle_recurrence(n, K, inf, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if ok != 1:
        return None
    return tuple(int(v) for v in out)


def apsp(W: np.ndarray, inf: int = INF16) -> np.ndarray:
    """min(shortest path weight, inf) for every ordered pair, by Floyd-Warshall
    relaxation (non-negative weights, inf = no arc)."""
    W = np.ascontiguousarray(W, dtype=np.int32)
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("W must be square")
    D = np.empty_like(W)
    _load().oracle_apsp(W.shape[0], _i32(W), inf, _i32(D))
    return D


def constant_difference(X: np.ndarray, Y: np.ndarray, inf: int = INF16):
    """(holds, b) of Algorithm 3's test: X = b (x) Y exactly, i.e. the same INF
    entries and one common difference b over the finite ones (b = 0 when no
    entry is finite)."""
    X = np.ascontiguousarray(X, dtype=np.int32)
    Y = np.ascontiguousarray(Y, dtype=np.int32)
    if X.shape != Y.shape:
        raise ValueError("X and Y must have one shape")
    b = ctypes.c_int64(0)
    ok = _load().oracle_constant_difference(X.size, _i32(X), _i32(Y), inf, ctypes.byref(b))
    return bool(ok), int(b.value)


# -- columns that are copies of the cycle (small cycle, any path) -----------

def cyclic_word_count(m: int) -> int:
    """Number of correct cyclic words of length m (column C_m, m >= 3)."""
    r = int(_load().oracle_cyclic_words(m, None))
    if r < 0:
        raise ValueError("the cycle order m must be in 3..16")
    return r


def cyclic_words(m: int) -> np.ndarray:
    """Base-3 codes of the correct cyclic words, increasing."""
    N = cyclic_word_count(m)
    out = np.zeros(N, dtype=np.uint32)
    _load().oracle_cyclic_words(m, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def is_correct_cyclic_word(m: int, code: int) -> bool:
    return bool(_load().oracle_is_correct_cyclic_word(m, code))


def cyclic_follows(m: int, q: int, p: int) -> bool:
    """True when cyclic word p can follow cyclic word q along the path."""
    return bool(_load().oracle_cyclic_follows(m, q, p))


def cyclic_can_start(m: int, p: int) -> bool:
    return bool(_load().oracle_cyclic_can_start(m, p))


def cyclic_can_end(m: int, p: int) -> bool:
    return bool(_load().oracle_cyclic_can_end(m, p))


def cyclic_state_matrix(m: int, inf: int = INF16) -> np.ndarray:
    """The column digraph's matrix for cyclic columns, N x N int32."""
    N = cyclic_word_count(m)
    A = np.empty((N, N), dtype=np.int32)
    _load().oracle_cyclic_state_matrix(m, inf, _i32(A))
    return A


def cyclic_boundary(m: int, inf: int = INF16):
    """(start, end) vectors of the open walk along the path, int32."""
    N = cyclic_word_count(m)
    s = np.empty(N, dtype=np.int32)
    e = np.empty(N, dtype=np.int32)
    _load().oracle_cyclic_boundary(m, inf, _i32(s), _i32(e))
    return s, e


def path_gamma2_sweep(m: int, nmax: int, inf: int = INF16) -> np.ndarray:
    """g[n-1] = gamma_2(P_n x C_m) for n = 1..nmax, by the vector chain over
    cyclic columns (start vector, then x <- x (x) A, end vector)."""
    if nmax < 1:
        raise ValueError("nmax must be at least 1")
    cyclic_word_count(m)
    g = np.empty(nmax, dtype=np.int32)
    _load().oracle_path_gamma2_sweep(m, nmax, inf, _i32(g))
    return g


def threads() -> int:
    """OpenMP threads the oracle's row-parallel loops use."""
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    """Threads for the oracle's later calls (timing only; results do not
    depend on it)."""
    _load().oracle_set_threads(int(t))


def brute_gamma2(n: int, m: int) -> int:
    """gamma_2(P_n x C_m) by exhaustive search (n*m <= 36)."""
    r = int(_load().brute_gamma2(n, m))
    if r < 0:
        raise ValueError("instance out of range for exhaustive search")
    return r


def brute_is_2dominating(n: int, m: int, mask: int) -> bool:
    return bool(_load().brute_is_2dominating(n, m, mask))
