"""The recurrence of the powers on the device (Algorithms 3, 4 and 5 with
Theorem 3) against the oracle, Tables 3 and 4, and the closed form; the
constant-difference kernel against the oracle's test."""
import sys

import numpy as np
import pytest

from closed_form import gamma2_closed_form
from conftest import read_table

pytestmark = pytest.mark.gpu

INF = 65535


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_17688_amd as tp
    return tp


@pytest.fixture(scope="module")
def tables():
    t3 = {int(r[0]): tuple(int(v) for v in r[1:]) for r in read_table("table3_recurrence.txt")}
    t4 = {int(r[0]): tuple(int(v) for v in r[1:]) for r in read_table("table4_min_recurrence.txt")}
    return t3, t4


def _padded(torch, M, ld):
    """M (int array, values <= INF) in a device u16 buffer with ld columns,
    the padding filled with a pattern that must not matter."""
    N = M.shape[0]
    buf = np.full((N, ld), 12345, dtype=np.uint16)
    buf[:, :N] = M.astype(np.uint16)
    t = torch.from_numpy(buf.view(np.int16)).cuda().view(torch.uint16)
    return t[:, :N]


def _holds(mm):
    mn, mx = int(mm[0]), int(mm[1])
    if mn == 2**31 - 1 and mx == -2**31:
        return True, 0
    return (mn == mx), (mn if mn == mx else None)


@pytest.mark.parametrize("N", [1, 7, 8, 37, 300, 1029])
def test_const_diff_matches_oracle(tp, oracle_mod, N):
    import torch
    rng = np.random.default_rng(N)
    ld = (N + 63) // 64 * 64
    Y = rng.integers(0, 600, (N, N)).astype(np.int64)
    Y[rng.random((N, N)) < 0.25] = INF
    Y[0, 0] = 7  # at least one finite entry
    shift = lambda M, b: np.where(M >= INF, INF, M + b)  # noqa: E731
    pairs = [(Y, Y), (shift(Y, 5), Y), (Y, shift(Y, 5))]
    fin = np.argwhere(Y < INF)
    i, j = fin[len(fin) // 2]
    X = shift(Y, 2)
    X[i, j] += 1
    pairs.append((X, Y))
    X = shift(Y, 2)
    X[i, j] = INF
    pairs.append((X, Y))
    full = np.full((N, N), INF)
    pairs.append((full, full))
    for c, (X, Yh) in enumerate(pairs):
        got = tp.tp_const_diff(_padded(torch, X, ld), _padded(torch, Yh, ld)).cpu().numpy()
        want = oracle_mod.constant_difference(X, Yh)
        holds, b = _holds(got)
        assert holds == want[0], (N, c, got)
        if holds:
            assert b == want[1], (N, c, got)
    assert _holds(tp.tp_const_diff(_padded(torch, shift(Y, 5), ld),
                                   _padded(torch, Y, ld)).cpu().numpy()) == (True, 5)


def test_const_diff_rejects_bad_arguments(tp):
    import torch
    X = torch.zeros((8, 8), dtype=torch.uint16, device="cuda")
    with pytest.raises(tp.TropicalError):
        tp.tp_const_diff(X, torch.zeros((8, 16), dtype=torch.uint16, device="cuda")[:, :8])
    with pytest.raises(TypeError):
        tp.tp_const_diff(X, torch.zeros((8, 8), dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("n", range(1, 10))
def test_recurrence_matches_oracle_and_tables(tp, oracle_mod, tables, n):
    say("recurrence", n)
    rec, diag = tp.tp_recurrence(n, 50)
    assert rec.K == 50 and rec.window == 49
    want = oracle_mod.recurrence(n, 50)
    if want is None:
        assert not rec.found
    else:
        assert rec.found and not rec.window_short
        assert (rec.r0, rec.a, rec.b, rec.n0) == want
    if n >= 2:
        t3, t4 = tables
        assert (rec.r0, rec.a, rec.b) == t3[n]
        assert (rec.n0, rec.a, rec.b) == t4[n]
    assert list(diag) == list(oracle_mod.gamma2_sweep(n, 50))


@pytest.mark.parametrize("n,window", [(10, 0), (11, 6), (12, 4)])
def test_recurrence_large_n_tables(tp, tables, n, window):
    say("recurrence", n, "window", window)
    rec, diag = tp.tp_recurrence(n, 50, window)
    t3, t4 = tables
    assert rec.found and not rec.window_short
    assert (rec.r0, rec.a, rec.b) == t3[n]
    assert (rec.n0, rec.a, rec.b) == t4[n]
    for m in range(3, 51):
        assert diag[m - 1] == gamma2_closed_form(n, m), (n, m)
    for m in range(3, 2001):
        assert tp.tp_gamma2_recurrence(rec, diag, m) == gamma2_closed_form(n, m), (n, m)


def test_gamma2_from_device_recurrence(tp, oracle_mod):
    # every n the oracle's long chains cover, any m up to 500 (Theorem 3 past K)
    for n in range(1, 9):
        rec, diag = tp.tp_recurrence(n, 50)
        long = oracle_mod.gamma2_sweep(n, 500)
        for m in range(3, 501):
            assert tp.tp_gamma2_recurrence(rec, diag, m) == long[m - 1], (n, m)
        for m in range(3, 3001, 7):
            assert tp.tp_gamma2_recurrence(rec, diag, m) == gamma2_closed_form(n, m), (n, m)


def test_window_short_and_window_enough(tp, tables):
    # n = 7 repeats at distance 18 (Table 3): a window of 10 cannot see it
    rec, _ = tp.tp_recurrence(7, 50, 10)
    assert rec.window == 10 and not rec.found and rec.window_short
    rec, _ = tp.tp_recurrence(7, 50, 18)
    t3, t4 = tables
    assert rec.found and (rec.r0, rec.a, rec.b) == t3[7] and rec.n0 == t4[7][0]


@pytest.mark.parametrize("n,K", [(4, 20), (6, 20), (7, 30), (8, 20), (8, 30), (9, 28), (2, 3)])
def test_short_chains_match_oracle(tp, oracle_mod, n, K):
    rec, diag = tp.tp_recurrence(n, K)
    want = oracle_mod.recurrence(n, K)
    if want is None:
        assert not rec.found and not rec.window_short
    else:
        assert rec.found and (rec.r0, rec.a, rec.b, rec.n0) == want
    assert list(diag) == list(oracle_mod.gamma2_sweep(n, K))


def test_recurrence_rejects_bad_arguments(tp):
    lib = tp.lib
    import ctypes
    rec = tp.Recurrence()
    diag = (ctypes.c_int32 * 64)()
    assert lib.tp_recurrence(0, 50, 0, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(14, 50, 0, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(5, 1, 0, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(5, 50, -1, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(5, 50, 0, None, diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(5, 70000, 0, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(5, 50, 257, ctypes.byref(rec), diag, None) == tp.TP_EINVAL
    assert lib.tp_recurrence(12, 6000, 0, ctypes.byref(rec), diag, None) == tp.TP_EOVERFLOW


def test_n13_beyond_the_papers_gpu(tp):
    """n = 13 (N = 131,562; 34.6 GB per power, which the paper could not fit):
    parity unpinned, so only properties.  Lemma 1 read on the diagonal: once
    the powers repeat with (a, b) from n0 on, so do their diagonal minima;
    Theorem 3's solution agrees with the computed minima; and the paper's
    conjecture gamma_2 = (n + 2) m / 3 for m = 0 (mod 3) (Section 4), and the
    one proven value Section 4 quotes for this path order: 2n + 1 = 27 at
    cycle 5."""
    say("recurrence 13")
    rec, diag = tp.tp_recurrence(13, 50, 3)
    assert rec.K == 50 and rec.window == 3
    if rec.found:
        for m in range(rec.n0, 51 - rec.a):
            assert diag[m + rec.a - 1] == diag[m - 1] + rec.b, m
        for m in range(3, 51):
            assert tp.tp_gamma2_recurrence(rec, diag, m) == diag[m - 1]
    for m in range(3, 51, 3):
        assert diag[m - 1] == 15 * m // 3, m
    # the cycle-5 value the paper quotes from its companion work (Section 4):
    # gamma_2(C_5 x P_n) = 2n + 1 for odd n, proven for every path order
    assert diag[5 - 1] == 2 * 13 + 1


@pytest.mark.parametrize("n,K,window", [(1, 50, 0), (2, 50, 0), (4, 50, 0), (6, 50, 0),
                                        (7, 50, 10), (7, 50, 18), (8, 50, 0), (9, 50, 0),
                                        (10, 50, 0), (8, 5, 0), (5, 4, 0)])
def test_compact_chain_recurrence_matches_16_bits(tp, oracle_mod, n, K, window):
    """The chain on shared-base compact powers (forced from n = 2 on) gives
    the 16-bit chain's search results and diagonal minima, and the oracle's."""
    say("compact recurrence", n, K, window)
    try:
        tp.tp_tune_compact_chains(0)
        rec16, diag16 = tp.tp_recurrence(n, K, window)
        tp.tp_tune_compact_chains(2)
        rec8, diag8 = tp.tp_recurrence(n, K, window)
    finally:
        tp.tp_tune_compact_chains(11)
    fields = ("K", "window", "found", "window_short", "r0", "a", "b", "n0")
    assert [getattr(rec8, f) for f in fields] == [getattr(rec16, f) for f in fields]
    assert list(diag8) == list(diag16) == list(oracle_mod.gamma2_sweep(n, K))
    want = oracle_mod.recurrence(n, K)
    if want is not None and not rec8.window_short:
        assert (rec8.r0, rec8.a, rec8.b, rec8.n0) == want


@pytest.mark.parametrize("n,K,window", [(11, 200, 6), (12, 120, 4)])
def test_compact_chain_long_runs_closed_form(tp, tables, n, K, window):
    """Long chains on shared-base compact powers (the default from n = 11):
    every diagonal minimum up to K == the closed form, and the recurrence of
    Tables 3 and 4 found at i = K."""
    say("long compact recurrence", n, K, window)
    rec, diag = tp.tp_recurrence(n, K, window)
    t3, t4 = tables
    assert rec.found and not rec.window_short
    assert rec.r0 == K - rec.a and (rec.a, rec.b) == t3[n][1:]
    assert (rec.n0, rec.a, rec.b) == t4[n]
    for m in range(3, K + 1):
        assert diag[m - 1] == gamma2_closed_form(n, m), (n, m)
