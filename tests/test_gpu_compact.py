"""Compact powers (8-bit residuals with one offset per row): the chain step,
the conversions and the diagonal minimum against the oracle's powers, the
16-bit chain and the closed form."""
import numpy as np
import pytest

import synth

from closed_form import gamma2_closed_form

pytestmark = pytest.mark.gpu

INF = 65535


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_17688_amd as tp
    return tp


def _dev16(M):
    import torch
    return torch.from_numpy(np.ascontiguousarray(M, dtype=np.uint16).view(np.int16)).cuda() \
        .view(torch.uint16)


def _host(T):
    return T.cpu().view(__import__("torch").int16).numpy().view(np.uint16).astype(np.int64)


def _u8(N, ncols):
    import torch
    return torch.empty((N, (ncols + 63) // 64 * 64 or 64), dtype=torch.uint8, device="cuda")


def _status():
    import torch
    return torch.zeros(1, dtype=torch.int32, device="cuda")


def _padded16(N, ncols=None):
    import torch
    ncols = N if ncols is None else ncols
    ld = (ncols + 63) // 64 * 64 or 64
    return torch.empty((N, ld), dtype=torch.uint16, device="cuda")[:, :ncols]


@pytest.mark.parametrize("n", range(2, 8))
def test_compact_chain_matches_oracle_powers(tp, oracle_mod, n):
    """A^k for k = 3..24 through compact steps == the oracle's A^k, and the
    compact diagonal minimum == the oracle's (Theorem 2)."""
    import torch
    A = oracle_mod.state_matrix(n)
    N = A.shape[0]
    P = [None, A]
    for _ in range(2, 25):
        P.append(oracle_mod.minplus(A, P[-1]))
    X8, Y8 = _u8(N, N), _u8(N, N)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(_dev16(P[3]), X8, RX, st)
    assert int(st.item()) == 0, n
    for k in range(3, 25):
        got = _host(tp.tp_compact_to_u16(X8, RX, N))
        assert (got == P[k]).all(), (n, k)
        assert tp.tp_compact_diag_min(X8[:, :N], RX) == oracle_mod.trace_min(P[k]), (n, k)
        tp.tp_compact_step(n, X8, RX, N, Y8, RY, st)
        X8, Y8, RX, RY = Y8, X8, RY, RX
    assert int(st.item()) == 0, n


@pytest.mark.parametrize("n,ncols,unroll", [(8, 1386, 4), (8, 1386, 8), (8, 700, 4),
                                            (8, 13, 8), (9, 3447, 4), (10, 1031, 8)])
def test_compact_chain_matches_u16_chain(tp, n, ncols, unroll):
    """Column panels of A^4, several 512-column panels and ragged tails:
    six compact steps == six 16-bit steps, element for element."""
    import torch
    N = tp.tp_state_dim(n)
    A = _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=A)
    X, Y = _padded16(N, ncols), _padded16(N, ncols)
    tp.tp_state_left_mul(n, A[:, :ncols].contiguous(), Y)  # A^2 on the columns
    tp.tp_state_left_mul(n, Y, X)
    tp.tp_state_left_mul(n, X, Y)
    X.copy_(Y)  # A^4 on the columns
    X8, Y8 = _u8(N, ncols), _u8(N, ncols)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(X, X8, RX, st)
    assert int(st.item()) == 0
    tp.tp_tune_compact_step(unroll)
    try:
        for k in range(6):
            tp.tp_state_left_mul(n, X, Y)
            X, Y = Y, X
            tp.tp_compact_step(n, X8, RX, ncols, Y8, RY, st)
            X8, Y8, RX, RY = Y8, X8, RY, RX
            assert torch.equal(tp.tp_compact_to_u16(X8, RX, ncols), X), (n, ncols, k)
    finally:
        tp.tp_tune_compact_step(0)
    assert int(st.item()) == 0


def test_compact_diag_min_gives_closed_form(tp):
    """gamma2(P_10 x C_m) for m = 3..40 as compact diagonal minima."""
    import torch
    n = 10
    N = tp.tp_state_dim(n)
    A, B = _padded16(N), _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=A)
    tp.tp_state_left_mul(n, A, B)
    tp.tp_state_left_mul(n, B, A)  # A^3
    X8, Y8 = _u8(N, N), _u8(N, N)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(A, X8, RX, st)
    for m in range(3, 41):
        assert tp.tp_compact_diag_min(X8[:, :N], RX) == gamma2_closed_form(n, m), m
        tp.tp_compact_step(n, X8, RX, N, Y8, RY, st)
        X8, Y8, RX, RY = Y8, X8, RY, RX
    assert int(st.item()) == 0


def test_compact_full_size_n12(tp):
    """n = 12 (N = 52,929), the size the step is measured at: two compact
    steps from A^3 == two 16-bit steps, every element."""
    import torch
    n = 12
    N = tp.tp_state_dim(n)
    X, Y = _padded16(N), _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=X)
    tp.tp_state_left_mul(n, X, Y)
    tp.tp_state_left_mul(n, Y, X)  # A^3
    X8, Y8 = _u8(N, N), _u8(N, N)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(X, X8, RX, st)
    assert int(st.item()) == 0
    for k in (4, 5):
        tp.tp_state_left_mul(n, X, Y)
        X, Y = Y, X
        tp.tp_compact_step(n, X8, RX, N, Y8, RY, st)
        X8, Y8, RX, RY = Y8, X8, RY, RX
        assert torch.equal(tp.tp_compact_to_u16(X8, RX, N), X), k
        assert tp.tp_compact_diag_min(X8[:, :N], RX) == tp.tp_trace_min(X), k
    assert int(st.item()) == 0


def test_compact_n13_column_panel(tp):
    """n = 13 (N = 131,562, successors past 2^16): a 1,000-column panel of
    A^3, three compact steps == three 16-bit steps."""
    import torch
    n, ncols = 13, 1000
    N = tp.tp_state_dim(n)
    idx = torch.arange(ncols, dtype=torch.int32, device="cuda") * 131
    X = tp.tp_build_state_columns(n, idx)
    Y = torch.empty_like(X)
    # A^3 columns: A x (A x columns of A)
    _left13(tp, n, X, Y)
    _left13(tp, n, Y, X)
    X8, Y8 = _u8(N, ncols), _u8(N, ncols)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(X, X8, RX, st)
    assert int(st.item()) == 0
    for k in range(3):
        _left13(tp, n, X, Y)
        X, Y = Y, X
        tp.tp_compact_step(n, X8, RX, ncols, Y8, RY, st)
        X8, Y8, RX, RY = Y8, X8, RY, RX
        assert torch.equal(tp.tp_compact_to_u16(X8, RX, ncols), X), k
    assert int(st.item()) == 0


def _left13(tp, n, X, Y):
    """Y = A(D_n) x X in 16 bits by the CSR product (tp_state_left_mul
    takes n <= 12)."""
    rowptr, col, z = tp.tp_build_state_csr(n)
    tp.tp_minplus_spmm(rowptr, col, z, X, Y)


def test_compact_conversion_reports_what_it_cannot_hold(tp, oracle_mod):
    import torch
    # A itself: rows with finite and INF entries
    A = oracle_mod.state_matrix(5)
    N = A.shape[0]
    st = _status()
    tp.tp_compact_from_u16(_dev16(A), _u8(N, N), torch.empty(N, dtype=torch.int32,
                                                              device="cuda"), st)
    assert int(st.item()) & tp.COMPACT_MIXED
    # a row spanning 300
    M = np.zeros((4, 40), dtype=np.int64)
    M[2, 7] = 300
    st = _status()
    tp.tp_compact_from_u16(_dev16(M), _u8(4, 40), torch.empty(4, dtype=torch.int32,
                                                               device="cuda"), st)
    assert int(st.item()) == tp.COMPACT_RANGE
    # spans of exactly 254 and rows of INF only are held and come back unchanged
    M = np.full((5, 77), 1000, dtype=np.int64)
    M[0, 3] = 1254
    M[1, :] = INF
    M[3, :] = np.arange(77) + 60000
    st = _status()
    X8 = _u8(5, 77)
    R = torch.empty(5, dtype=torch.int32, device="cuda")
    tp.tp_compact_from_u16(_dev16(M), X8, R, st)
    assert int(st.item()) == 0
    assert int(R[1].item()) == tp.COMPACT_DEAD
    assert (_host(tp.tp_compact_to_u16(X8, R, 77)) == M).all()


def test_compact_step_with_dead_rows(tp):
    """Rows of INF only in the input (dead successors) give the 16-bit step's
    result."""
    import torch
    n = 7
    N = tp.tp_state_dim(n)
    A, B = _padded16(N), _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=A)
    tp.tp_state_left_mul(n, A, B)
    tp.tp_state_left_mul(n, B, A)  # A^3
    rng = np.random.default_rng(7)
    dead = torch.from_numpy(rng.random(N) < 0.3).cuda()
    A.view(torch.int16)[dead] = -1  # INF
    X8, Y8 = _u8(N, N), _u8(N, N)
    RX = torch.empty(N, dtype=torch.int32, device="cuda")
    RY = torch.empty_like(RX)
    st = _status()
    tp.tp_compact_from_u16(A, X8, RX, st)
    assert int(st.item()) == 0
    tp.tp_state_left_mul(n, A, B)
    tp.tp_compact_step(n, X8, RX, N, Y8, RY, st)
    assert torch.equal(tp.tp_compact_to_u16(Y8, RY, N), B)
    assert int(st.item()) == 0


def test_compact_argument_checks(tp):
    import torch
    n = 4
    N = tp.tp_state_dim(n)
    X8, Y8 = _u8(N, N), _u8(N, N)
    R = torch.zeros(N, dtype=torch.int32, device="cuda")
    R2 = torch.zeros(N, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        tp.tp_compact_step(n, X8, R, N, X8, R2)  # in place
    odd = torch.empty((N, 60), dtype=torch.uint8, device="cuda")[:, :N]
    with pytest.raises(RuntimeError):
        tp.tp_compact_step(n, odd, R, N, Y8, R2)  # ld not a multiple of 8
    with pytest.raises(RuntimeError):
        tp.tp_compact_step(14, X8, R, N, Y8, R2)
    tp.tp_compact_step(n, X8, R, 0, Y8, R2)  # no columns: nothing to do
    with pytest.raises(RuntimeError):
        tp.tp_tune_compact_step(5)


# ------------------------------------------------------ shared-base form --

def _base2():
    import torch
    return torch.empty(2, dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("n", range(2, 8))
def test_shared_chain_matches_oracle_powers(tp, oracle_mod, n):
    """A^k, k = 3..40, through shared-base steps == the oracle's A^k, with
    the diagonal minima."""
    A = oracle_mod.state_matrix(n)
    N = A.shape[0]
    P = [None, A]
    for _ in range(2, 41):
        P.append(oracle_mod.minplus(A, P[-1]))
    X8, Y8, bx, by, st = _u8(N, N), _u8(N, N), _base2(), _base2(), _status()
    tp.tp_compact_shared_from_u16(_dev16(P[3]), X8, bx, st)
    assert int(st.item()) == 0, n
    for k in range(3, 41):
        assert (_host(tp.tp_compact_shared_to_u16(X8, bx, N)) == P[k]).all(), (n, k)
        assert tp.tp_compact_shared_diag_min(X8[:, :N], bx) == oracle_mod.trace_min(P[k]), (n, k)
        tp.tp_compact_shared_step(n, X8, bx, N, Y8, by, st)
        X8, Y8, bx, by = Y8, X8, by, bx
    assert int(st.item()) == 0, n


@pytest.mark.parametrize("n,ncols,unroll", [(8, 1386, 4), (8, 700, 8), (8, 13, 4),
                                            (9, 3447, 8), (11, 2100, 4), (8, 1386, 0x104),
                                            (8, 13, 0x108), (9, 3447, 0x104), (11, 2100, 0x108),
                                            (12, 600, 0x104)])
def test_shared_chain_matches_u16_chain(tp, n, ncols, unroll):
    """Chains of the shared-base step (entry at a time, 4 or 8 per round, or
    a mask group at a time: 0x100 | U) equal the 16-bit chain."""
    import torch
    N = tp.tp_state_dim(n)
    A = _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=A)
    X, Y = _padded16(N, ncols), _padded16(N, ncols)
    tp.tp_state_left_mul(n, A[:, :ncols].contiguous(), Y)
    tp.tp_state_left_mul(n, Y, X)  # A^3 on the columns
    X8, Y8, bx, by, st = _u8(N, ncols), _u8(N, ncols), _base2(), _base2(), _status()
    tp.tp_compact_shared_from_u16(X, X8, bx, st)
    assert int(st.item()) == 0
    tp.tp_tune_compact_step(unroll)
    try:
        for k in range(8):
            tp.tp_state_left_mul(n, X, Y)
            X, Y = Y, X
            tp.tp_compact_shared_step(n, X8, bx, ncols, Y8, by, st)
            X8, Y8, bx, by = Y8, X8, by, bx
            assert torch.equal(tp.tp_compact_shared_to_u16(X8, bx, ncols), X), (n, ncols, k)
    finally:
        tp.tp_tune_compact_step(0)
    assert int(st.item()) == 0


def test_shared_full_size_n12_and_closed_form(tp):
    """n = 12 at full size: three shared-base steps from A^3 == the 16-bit
    steps, and the diagonal minima == the closed form."""
    import torch
    n = 12
    N = tp.tp_state_dim(n)
    X, Y = _padded16(N), _padded16(N)
    tp.tp_build_state_matrix(n, tp.TP_U16, out=X)
    tp.tp_state_left_mul(n, X, Y)
    tp.tp_state_left_mul(n, Y, X)  # A^3
    X8, Y8, bx, by, st = _u8(N, N), _u8(N, N), _base2(), _base2(), _status()
    tp.tp_compact_shared_from_u16(X, X8, bx, st)
    assert int(st.item()) == 0
    for m in (4, 5, 6):
        tp.tp_state_left_mul(n, X, Y)
        X, Y = Y, X
        tp.tp_compact_shared_step(n, X8, bx, N, Y8, by, st)
        X8, Y8, bx, by = Y8, X8, by, bx
        assert torch.equal(tp.tp_compact_shared_to_u16(X8, bx, N), X), m
        assert tp.tp_compact_shared_diag_min(X8[:, :N], bx) == gamma2_closed_form(n, m), m
    assert int(st.item()) == 0


def test_shared_conversion_reports(tp, oracle_mod):
    A = oracle_mod.state_matrix(5)
    N = A.shape[0]
    st = _status()
    tp.tp_compact_shared_from_u16(_dev16(A), _u8(N, N), _base2(), st)
    assert int(st.item()) & tp.COMPACT_MIXED
    M = np.full((6, 50), 500, dtype=np.int64)
    M[4, 9] = 755
    st = _status()
    tp.tp_compact_shared_from_u16(_dev16(M), _u8(6, 50), _base2(), st)
    assert int(st.item()) == tp.COMPACT_RANGE
    M[4, 9] = 754
    st, X8, b = _status(), _u8(6, 50), _base2()
    tp.tp_compact_shared_from_u16(_dev16(M), X8, b, st)
    assert int(st.item()) == 0
    assert b.tolist() == [500, 0]
    assert (_host(tp.tp_compact_shared_to_u16(X8, b, 50)) == M).all()


def test_shared_argument_checks(tp):
    import torch
    n = 4
    N = tp.tp_state_dim(n)
    X8, Y8 = _u8(N, N), _u8(N, N)
    b1, b2 = _base2(), _base2()
    with pytest.raises(RuntimeError):
        tp.tp_compact_shared_step(n, X8, b1, N, X8, b2)  # in place
    with pytest.raises(RuntimeError):
        tp.tp_compact_shared_step(n, X8, b1, N, Y8, b1)  # one base word for both
    odd = torch.empty((N, 60), dtype=torch.uint8, device="cuda")[:, :N]
    with pytest.raises(RuntimeError):
        tp.tp_compact_shared_step(n, odd, b1, N, Y8, b2)  # ld not a multiple of 8
    with pytest.raises(RuntimeError):
        tp.tp_compact_shared_step(0, X8, b1, N, Y8, b2)
    with pytest.raises(RuntimeError):
        tp.tp_tune_compact_chains(-1)
    tp.tp_compact_shared_step(n, X8, b1, 0, Y8, b2)  # no columns: nothing to do
    # an empty matrix converts to base {INF, 0} and no status
    st = _status()
    Y, b = tp.tp_compact_shared_from_u16(_dev16(np.zeros((0, 0), dtype=np.int64)), status=st)
    assert b.tolist() == [INF, 0] and int(st.item()) == 0


@pytest.mark.parametrize("N,count,ld_pad", [(1, 1, 64), (63, 63, 64), (64, 20, 64), (65, 65, 3),
                                            (225, 100, 64), (1000, 1000, 8), (1000, 333, 64),
                                            (2100, 777, 16)])
def test_shared_select_trace_vs_oracle(tp, oracle_mod, N, count, ld_pad):
    """Trace of X x P on selected diagonal entries == the oracle's product of
    the listed rows of X with the panel P, read on its diagonal; with and
    without a row list, aligned (vector) and unaligned layouts, ragged t and
    k tiles."""
    import torch
    rng = np.random.default_rng(N + count)
    x, wx, _ = synth.residual_matrix(N, N, N, 0, 200, 900)
    p, wp, _ = synth.residual_matrix(N, count, N + 1, 2, 250, 31000)
    for use_idx in (False, True):
        if use_idx:
            idx = rng.choice(N, count, replace=count > N // 2).astype(np.int32)
        else:
            if count != N:
                continue
            idx = np.arange(N, dtype=np.int32)
        vals_x = x.astype(np.int32) + int(wx[0])
        vals_p = p.astype(np.int32) + int(wp[0])
        prod = oracle_mod.minplus(vals_x[idx], vals_p)
        ref = min(oracle_mod.trace_min(prod), INF)
        ldx = (N + ld_pad - 1) // ld_pad * ld_pad
        ldp = (count + ld_pad - 1) // ld_pad * ld_pad
        X8 = torch.zeros((N, ldx), dtype=torch.uint8, device="cuda")
        P8 = torch.zeros((N, ldp), dtype=torch.uint8, device="cuda")
        X8[:, :N] = torch.from_numpy(x).cuda()
        P8[:, :count] = torch.from_numpy(p).cuda()
        bx, bp = torch.from_numpy(wx).cuda(), torch.from_numpy(wp).cuda()
        di = torch.from_numpy(idx).cuda() if use_idx else None
        got = int(tp.tp_compact_shared_select_trace(X8, bx, P8[:, :count], bp, di).item())
        assert got == ref, (N, count, ld_pad, use_idx)
        # saturation: bases whose sum passes INF give INF
        big = torch.tensor([40000, 0], dtype=torch.int32, device="cuda")
        got = int(tp.tp_compact_shared_select_trace(X8, big, P8[:, :count], big, di).item())
        assert got == INF


def test_shared_select_trace_arguments(tp):
    import torch
    X8 = torch.zeros((10, 16), dtype=torch.uint8, device="cuda")
    b = torch.zeros(2, dtype=torch.int32, device="cuda")
    out = tp.tp_compact_shared_select_trace(X8[:0, :0], b, X8[:0, :0], b)
    assert int(out.item()) == INF  # no entry: INF
    f = tp.lib.tp_compact_shared_select_trace
    p, pb, po = X8.data_ptr(), b.data_ptr(), out.data_ptr()
    assert f(10, 11, None, p, 16, pb, p, 16, pb, po, None) == tp.TP_EINVAL  # count > N, no list
    assert f(10, 10, None, p, 9, pb, p, 16, pb, po, None) == tp.TP_EINVAL   # ldx < N
    assert f(10, 10, None, p, 16, pb, p, 16, None, po, None) == tp.TP_EINVAL
    assert f(10, 10, None, p, 16, pb, p, 16, pb, None, None) == tp.TP_EINVAL
