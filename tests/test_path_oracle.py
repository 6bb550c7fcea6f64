"""The oracle's small-cycle / any-path construction against what fixes it.

Columns are copies of the cycle C_m and the walk runs along the path P_n
(the complementary problem Section 1 names, on the column construction of
Section 2.1 with the labelling rules of Section 2.2 read around the cycle).
The references are independent of that construction: exhaustive search from
the definition of 2-domination, the paper's own construction (columns are
copies of the path, closed walks around the cycle: the same graph), the
closed form of Section 4 (Tables 4 and 6), the formulas Section 4 quotes from
its companion work for cycles 3, 5 and 6, the textbook value of a cycle, and a
transfer-matrix count of the cyclic words.
"""
import itertools

import numpy as np
import pytest

from closed_form import gamma2_closed_form

INF = 65535


def _letters(m, code):
    out = []
    for _ in range(m):
        out.append(code % 3)
        code //= 3
    return out[::-1]


def _code(word):
    c = 0
    for ch in word:
        c = 3 * c + int(ch)
    return c


def test_cyclic_word_counts_by_transfer_matrix(oracle_mod):
    """|cyclic words of length m| = trace(T^m), T the 9 x 9 transfer matrix on
    letter pairs (a, b) -> (b, c) allowed when the window abc breaks neither
    column rule (no 020, no nonzero-1-nonzero)."""
    def ok(a, b, c):
        return not (b == 2 and a == 0 and c == 0) and not (b == 1 and a != 0 and c != 0)
    T = np.zeros((9, 9), dtype=object)
    for a, b, c in itertools.product(range(3), repeat=3):
        if ok(a, b, c):
            T[3 * a + b, 3 * b + c] = 1
    P = np.identity(9, dtype=object)
    for m in range(1, 15):
        P = P.dot(T)
        if m >= 3:
            assert oracle_mod.cyclic_word_count(m) == int(np.trace(P)), m


def test_cyclic_rules_by_hand(oracle_mod):
    """Single words and pairs checked by hand for m = 4 (letters around the
    cycle, so the first and the last letter are neighbours)."""
    m = 4
    # 1 at position 1 with neighbours 0 (position 4, by the wrap) and 0
    assert oracle_mod.is_correct_cyclic_word(m, _code("1000"))
    # 2 at position 1 between two zeros, one of them through the wrap
    assert not oracle_mod.is_correct_cyclic_word(m, _code("2010"))
    # 2s at positions 1 and 4 next to each other, a 1 beside a 0
    assert oracle_mod.is_correct_cyclic_word(m, _code("2012"))
    # 1 at position 4 between a 2 and a 1 (position 1, by the wrap)
    assert not oracle_mod.is_correct_cyclic_word(m, _code("1021"))
    # start: each 1 of "0101" sees two zeros in its column
    assert oracle_mod.cyclic_can_start(m, _code("0101"))
    # start: each 2 of "0022" sees exactly one zero in its column
    assert oracle_mod.cyclic_can_start(m, _code("0022"))
    # start: in "0011" each 1 sees one zero only
    assert oracle_mod.is_correct_cyclic_word(m, _code("0011"))
    assert not oracle_mod.cyclic_can_start(m, _code("0011"))
    assert not oracle_mod.is_correct_cyclic_word(m, _code("0111"))
    # after "1100" each 1 of "0011" has its second zero in the column before
    assert oracle_mod.cyclic_follows(m, _code("1100"), _code("0011"))
    # after "1101" the 1 at position 4 has one zero only
    assert not oracle_mod.cyclic_follows(m, _code("1101"), _code("0011"))
    # a 2 in the column before forces a 0 beside it
    assert not oracle_mod.cyclic_follows(m, _code("2012"), _code("1010"))
    assert oracle_mod.cyclic_follows(m, _code("2012"), _code("0100"))
    # end: no 2
    assert oracle_mod.cyclic_can_end(m, _code("0101"))
    assert not oracle_mod.cyclic_can_end(m, _code("0022"))


def test_state_matrix_labels_and_boundary(oracle_mod):
    """Arcs carry the zeros of the successor; start carries the zeros of the
    first column; end is 0 or INF."""
    for m in (3, 4, 5):
        w = oracle_mod.cyclic_words(m)
        A = oracle_mod.cyclic_state_matrix(m)
        s, e = oracle_mod.cyclic_boundary(m)
        for j, c in enumerate(w):
            z = _letters(m, int(c)).count(0)
            col = A[:, j]
            assert set(col[col < INF].tolist()) <= {z}
            assert s[j] in (z, INF)
            assert e[j] in (0, INF)
            assert (e[j] == 0) == (2 not in _letters(m, int(c)))


def test_cycle_textbook(oracle_mod):
    """n = 1: the path of one vertex leaves the cycle, gamma_2(C_m) = ceil(m/2)."""
    for m in range(3, 10):
        assert oracle_mod.path_gamma2_sweep(m, 1)[0] == (m + 1) // 2, m


@pytest.mark.parametrize("m,nmax", [(3, 9), (4, 7), (5, 5), (6, 4), (7, 4), (8, 3)])
def test_exhaustive_search(oracle_mod, m, nmax):
    """gamma_2(P_n x C_m) against exhaustive search from the definition."""
    g = oracle_mod.path_gamma2_sweep(m, nmax)
    for n in range(1, nmax + 1):
        assert g[n - 1] == oracle_mod.brute_gamma2(n, m), (n, m)


def test_same_graph_other_construction(oracle_mod):
    """P_n x C_m is one graph whichever factor the columns copy: the walk along
    the path over cyclic columns equals the closed walk around the cycle over
    path columns (Theorem 2), n = 1..8, m = 3..10."""
    closed = {n: oracle_mod.gamma2_sweep(n, 10) for n in range(1, 9)}
    for m in range(3, 11):
        g = oracle_mod.path_gamma2_sweep(m, 8)
        for n in range(1, 9):
            assert g[n - 1] == closed[n][m - 1], (n, m)


def test_closed_form_paths_up_to_12(oracle_mod):
    """Section 4's closed form (Tables 4 and 6, cycle-5 exceptions) for every
    path order n <= 12 at cycles m = 3..9."""
    for m in range(3, 10):
        g = oracle_mod.path_gamma2_sweep(m, 12)
        for n in range(1, 13):
            assert g[n - 1] == gamma2_closed_form(n, m), (n, m)


def test_cycle5_formula_long_paths(oracle_mod):
    """The cycle-5 formula Section 4 quotes from the companion work:
    gamma_2(C_5 x P_n) = 2n + 2 for even n > 2, 2n + 1 for n = 2 or odd n."""
    g = oracle_mod.path_gamma2_sweep(5, 400)
    for n in range(2, 401):
        assert g[n - 1] == (2 * n + 2 if n > 2 and n % 2 == 0 else 2 * n + 1), n


@pytest.mark.parametrize("m", [3, 6, 9])
def test_multiple_of_three_long_paths(oracle_mod, m):
    """Section 4: the companion work obtained (n + 2) m / 3 for cycles of order
    3, 6, 9, 12, 15 and paths of order n >= 8."""
    nmax = 300 if m < 9 else 60
    g = oracle_mod.path_gamma2_sweep(m, nmax)
    for n in range(8, nmax + 1):
        assert g[n - 1] == (n + 2) * m // 3, (n, m)


def test_argument_checks(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.cyclic_word_count(2)
    with pytest.raises(ValueError):
        oracle_mod.path_gamma2_sweep(4, 0)
