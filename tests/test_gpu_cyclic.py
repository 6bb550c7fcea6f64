"""Small cycle, any path on the GPU: the cyclic column digraph, its boundary
vectors and the walk along the path, against the CPU oracle and the formulas
Section 4 quotes.

The oracle's construction (tests/test_path_oracle.py) is pinned against
exhaustive search, the paper's own construction of the same graph, the
closed form for n <= 12 and the cycle-5 and (n + 2) m / 3 formulas.  Here the
library's words, matrix (u8 and u16) and boundary vectors must equal the
oracle's element by element, and every form of the walk (one workgroup, a
launch per level, dense vector-matrix products, the plain per-query call)
must give the oracle's gamma_2 at every path order of the sweep.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2409_17688_amd as tp
    return tp


def host16(t):
    import torch
    torch.cuda.synchronize()
    if t.dtype == torch.uint16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.int64)
    return t.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("m", range(3, 13))
def test_words_and_counts(tp, oracle_mod, m):
    say("cyclic words", m)
    N = tp.tp_cyclic_dim(m)
    assert N == oracle_mod.cyclic_word_count(m)
    got = tp.tp_cyclic_words(m).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle_mod.cyclic_words(m))


@pytest.mark.parametrize("m", range(3, 10))
def test_matrix_and_boundary(tp, oracle_mod, m):
    """Dense matrix (u16 and u8, padded leading dimension), the arc count and
    the boundary vectors, bit-exact against the oracle."""
    import torch
    say("cyclic matrix", m)
    N = tp.tp_cyclic_dim(m)
    ref = oracle_mod.cyclic_state_matrix(m)
    A = tp.tp_build_cyclic_matrix(m, tp.TP_U16)
    assert np.array_equal(host16(A), ref)
    ref8 = np.where(ref >= 65535, 255, ref)
    big = torch.full((N, N + 37), 7, dtype=torch.uint8, device="cuda")
    tp.tp_build_cyclic_matrix(m, tp.TP_U8, big[:, :N])
    B = host16(big)
    assert np.array_equal(B[:, :N], ref8)
    assert (B[:, N:] == 7).all()
    assert tp.tp_cyclic_nnz(m) == int((ref < 65535).sum())
    s_ref, e_ref = oracle_mod.cyclic_boundary(m)
    for dt, inf in ((tp.TP_U16, 65535), (tp.TP_U8, 255)):
        s, e = tp.tp_build_cyclic_boundary(m, dt)
        assert np.array_equal(host16(s), np.where(s_ref >= 65535, inf, s_ref))
        assert np.array_equal(host16(e), np.where(e_ref >= 65535, inf, e_ref))


SWEEP = {3: 400, 4: 400, 5: 400, 6: 400, 7: 300, 8: 256, 9: 120, 10: 40}


@pytest.mark.parametrize("m", sorted(SWEEP))
def test_sweep_every_form_vs_oracle(tp, oracle_mod, m):
    """gamma_2(P_k x C_m), k = 1..nmax, from each form of the walk == the
    oracle's vector chain at every k."""
    nmax = SWEEP[m]
    say("cyclic sweep", m, nmax)
    ref = oracle_mod.path_gamma2_sweep(m, nmax)
    forms = [tp.TP_WALK_AUTO, tp.TP_WALK_STEPS, tp.TP_WALK_GEMV]
    if tp.tp_cyclic_dim(m) <= (65536 - 1024) // 6:
        forms.append(tp.TP_WALK_CHAIN)
    for form in forms:
        got = tp.tp_cyclic_walk_sweep(m, nmax, form=form).cpu().numpy()
        assert np.array_equal(got, ref), (m, form)


@pytest.mark.parametrize("m", [11, 12])
def test_sweep_large_cycles_closed_form(tp, m):
    """m = 11, 12 (N = 22,376 and 55,603): the sweep against Section 4's closed
    form with Tables 4 and 6 for every path order n <= 12 (the oracle's dense
    matrix would not fit the host at m = 12)."""
    from closed_form import gamma2_closed_form
    say("cyclic sweep large", m)
    got = tp.tp_cyclic_walk_sweep(m, 12).cpu().numpy()
    for n in range(1, 13):
        assert got[n - 1] == gamma2_closed_form(n, m), (n, m)
    assert tp.tp_cyclic_walk_gamma2(12, m) == gamma2_closed_form(12, m)


def test_cycle5_formula_long_paths(tp):
    """gamma_2(C_5 x P_n) = 2n + 2 for even n > 2, 2n + 1 for n = 2 or odd n
    (the formula Section 4 quotes from its companion work), n = 1..13000."""
    say("cycle 5 to 13000")
    nmax = 13000
    got = tp.tp_cyclic_walk_sweep(5, nmax).cpu().numpy()
    n = np.arange(1, nmax + 1)
    expect = np.where((n > 2) & (n % 2 == 0), 2 * n + 2, 2 * n + 1)
    expect[0] = 3  # n = 1: the cycle alone, ceil(5 / 2)
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("m", [3, 6, 9])
def test_multiple_of_three_long_paths(tp, m):
    """(n + 2) m / 3 for cycles 3, 6, 9 and paths n >= 8 (quoted in Section 4
    from the companion work), to n = 2000."""
    say("multiple of three", m)
    nmax = 2000
    got = tp.tp_cyclic_walk_sweep(m, nmax).cpu().numpy()
    for n in range(8, nmax + 1):
        assert got[n - 1] == (n + 2) * m // 3, (n, m)


@pytest.mark.parametrize("n,m", [(1, 3), (2, 4), (5, 5), (17, 6), (64, 7), (200, 8), (33, 9)])
def test_plain_walk_vs_oracle(tp, oracle_mod, n, m):
    """The per-query call (dense vector-matrix products) == the oracle."""
    say("plain walk", n, m)
    assert tp.tp_cyclic_walk_gamma2(n, m) == int(oracle_mod.path_gamma2_sweep(m, n)[n - 1])


def test_same_numbers_as_the_other_construction(tp):
    """The walk over cyclic columns and the closed walk over path columns
    (tp_tropical_power_trace, Theorem 2) give the same gamma_2 for one graph."""
    say("both constructions")
    for m in range(3, 9):
        sweep = tp.tp_cyclic_walk_sweep(m, 9).cpu().numpy()
        for n in range(1, 10):
            assert int(sweep[n - 1]) == tp.tp_tropical_power_trace(n, m), (n, m)


def test_argument_checks(tp):
    import torch
    say("argument checks")
    with pytest.raises(tp.TropicalError):
        tp.tp_cyclic_dim(2)
    with pytest.raises(tp.TropicalError):
        tp.tp_cyclic_dim(13)
    with pytest.raises(tp.TropicalError):
        tp.tp_cyclic_walk_gamma2(0, 5)
    with pytest.raises(tp.TropicalError) as e:
        tp.tp_cyclic_walk_gamma2(6554, 10)
    assert e.value.status == tp.TP_EOVERFLOW
    with pytest.raises(tp.TropicalError) as e:
        tp.tp_cyclic_walk_sweep(12, 5462)
    assert e.value.status == tp.TP_EOVERFLOW
    with pytest.raises(tp.TropicalError):
        tp.tp_cyclic_walk_sweep(11, 5, form=tp.TP_WALK_CHAIN)  # N = 22,376 does not fit
    with pytest.raises(tp.TropicalError):
        tp.tp_cyclic_walk_sweep(5, 5, form=7)
    # a bad dtype through the C ABI itself: rejected, nothing written
    A = torch.full((92, 92), 7, dtype=torch.uint8, device="cuda")
    assert tp.lib.tp_build_cyclic_matrix(5, 3, A.data_ptr(), 92, None) == tp.TP_EINVAL
    assert tp.lib.tp_build_cyclic_matrix(5, tp.TP_U8, A.data_ptr(), 91, None) == tp.TP_EINVAL
    out = torch.full((4,), -9, dtype=torch.int32, device="cuda")
    assert tp.lib.tp_cyclic_walk_sweep(5, 4, out.data_ptr(), 9, None) == tp.TP_EINVAL
    torch.cuda.synchronize()
    assert (A.cpu() == 7).all() and (out.cpu() == -9).all()
