"""The chain step at the path orders the default chains run on (n = 10..13),
against the CPU oracle on sampled rows.

A(D_n) is too large for the oracle to hold whole from n = 11 on (N = 21,294
and 52,929), so the oracle builds only the sampled rows of Algorithm 1's
matrix (``oracle.state_rows``, the same follows test as the whole matrix) and
multiplies them by the same X with its plain (min,+) product.  Every step
form the default path can take is compared element by element on those rows:
the 16-bit row-block step, the 16-bit per-row (CSR) step, the automatic
choice, and both compact forms (8-bit residuals over one offset per row, and
over one base per power) on the same values.  X spans two full 512-column
panels and a ragged tail; rows include the all-zero word (the longest
successor list), both ends of 16-row blocks and the last rows.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

NCOLS = 1100  # two 512-column panels and a ragged panel of 76 columns


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2409_17688_amd as tp
    return tp


def sample_rows(N, seed, count=64):
    fixed = [0, 1, 2, 15, 16, 17, N // 2, N - 17, N - 16, N - 2, N - 1]
    rng = np.random.default_rng(seed)
    rest = rng.choice(np.arange(3, N - 2), count - len(fixed), replace=False)
    return np.unique(np.concatenate([fixed, rest])).astype(np.int64)


def dev16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)).cuda() \
        .view(torch.uint16)


def padded(N, ncols, dtype):
    import torch
    ld = (ncols + 63) // 64 * 64
    return torch.empty((N, ld), dtype=dtype, device="cuda")[:, :ncols]


def rows_of(t, rows):
    import torch
    torch.cuda.synchronize()
    idx = torch.from_numpy(rows).cuda()
    if t.dtype == torch.uint16:
        # torch has no uint16 gather: the rows of the same bits viewed as int16
        r = t.view(torch.int16)[idx]
        return r.cpu().numpy().view(np.uint16).astype(np.int64)
    return t[idx].cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("n", [10, 11, 12, 13])
@pytest.mark.parametrize("dist", [(0, 30000, 0.3), (0, 40, 0.0), (65000, 65534, 0.0)])
def test_u16_step_sampled_rows_vs_oracle(tp, oracle_mod, n, dist):
    """Y = A(D_n) x X in 16 bits: the blocked, per-row and automatic steps,
    on unpadded and 64-entry padded rows, == the oracle on 64 sampled rows."""
    N = tp.tp_state_dim(n)
    rows = sample_rows(N, 300 + n)
    lo, hi, frac = dist
    say("u16 step vs oracle rows", n, dist)
    X = synth.stress_matrix(N, NCOLS, 400 + n, lo, hi, frac, np.uint16)
    ref = oracle_mod.minplus(oracle_mod.state_rows(n, rows), X.astype(np.int32))
    Xd = dev16(X)
    Xp = padded(N, NCOLS, Xd.dtype)
    Xp.copy_(Xd)
    forms = [tp.TP_STEP_BLOCKED, tp.TP_STEP_BLOCKED_ENTRIES, tp.TP_STEP_CSR, tp.TP_STEP_AUTO]
    for form in forms:
        for src in (Xd, Xp):
            Y = padded(N, NCOLS, Xd.dtype) if src is Xp else None
            Y = tp.tp_state_left_mul(n, src, Y, form=form)
            got = rows_of(Y, rows)
            assert np.array_equal(got, ref), (n, dist, form, src is Xp)
    del Xd, Xp


@pytest.mark.parametrize("n", [10, 11, 12, 13])
@pytest.mark.parametrize("lo,hi,base", [(0, 14, 600), (3, 40, 1234)])
def test_shared_base_step_sampled_rows_vs_oracle(tp, oracle_mod, n, lo, hi, base):
    """(Y, G_Y) = A(D_n) x (X, G_X) on shared-base compact powers (the default
    chain from n = 11): the values G_Y + y of 64 sampled rows == the oracle's
    product of the same rows with the values G_X + x."""
    import torch
    N = tp.tp_state_dim(n)
    rows = sample_rows(N, 500 + n)
    say("shared-base step vs oracle rows", n, lo, hi, base)
    x, word, _ = synth.residual_matrix(N, NCOLS, 600 + n, lo, hi, base)
    ref = oracle_mod.minplus(oracle_mod.state_rows(n, rows), x.astype(np.int32) + base)
    X8 = padded(N, NCOLS, torch.uint8)
    X8.copy_(torch.from_numpy(x).cuda())
    Y8 = padded(N, NCOLS, torch.uint8)
    bx = torch.from_numpy(word).cuda()
    by = torch.zeros(2, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for unroll in (4, 8, 4 | tp.TP_COMPACT_GROUPED, 8 | tp.TP_COMPACT_GROUPED):
        tp.tp_tune_compact_step(unroll)
        try:
            Y8.fill_(0xEE)
            tp.tp_compact_shared_step(n, X8, bx, NCOLS, Y8, by, st)
        finally:
            tp.tp_tune_compact_step(0)
        assert int(st.item()) == 0, (n, unroll)
        g = int(by[0].item())
        got = rows_of(Y8, rows) + g
        assert np.array_equal(got, ref), (n, lo, hi, base, unroll)
        # the output base is G_X + least residual, and no value is below it
        assert g == base + lo and int(by[1].item()) >= 0


@pytest.mark.parametrize("n", [10, 11, 12])
def test_per_row_compact_step_sampled_rows_vs_oracle(tp, oracle_mod, n):
    """(Y, R_Y) = A(D_n) x (X, R_X) on compact powers with one offset per row:
    R_Y[q] + y[q][c] of 64 sampled rows == the oracle's product of the same
    rows with the values R_X[p] + x[p][c]."""
    import torch
    N = tp.tp_state_dim(n)
    rows = sample_rows(N, 700 + n)
    say("per-row compact step vs oracle rows", n)
    x, _, off = synth.residual_matrix(N, NCOLS, 800 + n, 0, 30, 0, row_offsets=(400, 460))
    vals = x.astype(np.int32) + off[:, None]
    ref = oracle_mod.minplus(oracle_mod.state_rows(n, rows), vals)
    X8 = padded(N, NCOLS, torch.uint8)
    X8.copy_(torch.from_numpy(x).cuda())
    Y8 = padded(N, NCOLS, torch.uint8)
    RX = torch.from_numpy(off).cuda()
    RY = torch.empty_like(RX)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    tp.tp_compact_step(n, X8, RX, NCOLS, Y8, RY, st)
    assert int(st.item()) == 0, n
    got = rows_of(Y8, rows) + rows_of(RY, rows)[:, None]
    assert np.array_equal(got, ref), n
