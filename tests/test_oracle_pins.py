"""The CPU oracle against what the paper and the mathematics fix.

Each test names the passage it pins.  None of them compares the oracle with
itself: the references are printed tables, a hand-derived matrix, textbook
identities of the (min,+) semiring, exhaustive search from the definition of
2-domination, and the paper's closed forms.
"""
import numpy as np
import pytest

from closed_form import gamma2_closed_form
from conftest import read_table

INF = 65535


def test_word_counts_table1(oracle_mod):
    """Table 1: number of correct words for n = 2..13."""
    for n, rows, _mem in read_table("table1_rows.txt"):
        assert oracle_mod.word_count(int(n)) == int(rows), n


def test_n1_words_and_arcs(oracle_mod):
    """n = 1 (outside the paper, which starts at 2): words 0, 1, 2; the word 1
    needs two zeros but has only q_1 as a neighbour, so it has no in-arcs."""
    assert [oracle_mod.word_string(1, c) for c in oracle_mod.words(1)] == ["0", "1", "2"]
    A = oracle_mod.state_matrix(1)
    assert (A[:, 1] == INF).all()


def test_n2_matrix_hand_derived(oracle_mod):
    """Section 2.2 rules worked by hand for n = 2 (tests/golden/state_matrix_n2.txt)."""
    rows = read_table("state_matrix_n2.txt")
    names = rows[0]
    assert [oracle_mod.word_string(2, c) for c in oracle_mod.words(2)] == names
    expect = np.array([[INF if v == "I" else int(v) for v in r] for r in rows[1:]])
    A = oracle_mod.state_matrix(2)
    assert (A == expect).all()
    assert int((A < INF).sum()) == 15


def test_minplus_hand_example(oracle_mod):
    """Section 1 definition, a 2x3 by 3x2 product worked by hand (non-square,
    so a transposed operand cannot pass)."""
    I = INF
    A = np.array([[0, 3, I], [2, I, 1]])
    B = np.array([[1, I], [0, 4], [5, 2]])
    assert oracle_mod.minplus(A, B).tolist() == [[1, 7], [3, 3]]


def test_minplus_semiring_identities(oracle_mod):
    """Tropical identity, INF absorption, constant matrices and saturation."""
    rng = np.random.default_rng(1)
    X = rng.integers(0, 1000, size=(17, 23))
    X[rng.random(X.shape) < 0.3] = INF
    E = np.full((17, 17), INF)
    np.fill_diagonal(E, 0)
    assert (oracle_mod.minplus(E, X) == X).all()
    E2 = np.full((23, 23), INF)
    np.fill_diagonal(E2, 0)
    assert (oracle_mod.minplus(X, E2) == X).all()
    # an all-INF row on the left gives an all-INF row
    Y = X.copy()
    Y[3, :] = INF
    assert (oracle_mod.minplus(Y, rng.integers(0, 5, (23, 9)))[3] == INF).all()
    # right operand constant c: (X x C)_ij = min_k x_ik + c
    C = np.full((23, 5), 7)
    R = oracle_mod.minplus(X, C)
    assert (R == np.minimum(X.min(axis=1, keepdims=True) + 7, INF)).all()
    # saturation: sums >= INF are INF, INF - 1 stays finite
    S = oracle_mod.minplus(np.array([[INF - 2]]), np.array([[1, 2, 3]]))
    assert S.tolist() == [[INF - 1, INF, INF]]
    S8 = oracle_mod.minplus(np.array([[250]]), np.array([[4, 5, 200]]), inf=255)
    assert S8.tolist() == [[254, 255, 255]]
    # empty inner dimension gives INF
    Z = oracle_mod.minplus(np.zeros((2, 0), dtype=np.int32), np.zeros((0, 3), dtype=np.int32))
    assert (Z == INF).all()


def test_power_associativity(oracle_mod):
    """A^(a+b) = A^a x A^b in the exact integer semiring (Algorithm 2 powers)."""
    rng = np.random.default_rng(2)
    for n in (3, 4, 5, 6):
        for _ in range(3):
            a, b = (int(v) for v in rng.integers(1, 12, size=2))
            lhs = oracle_mod.power(n, a + b)
            rhs = oracle_mod.minplus(oracle_mod.power(n, a), oracle_mod.power(n, b))
            assert (lhs == rhs).all(), (n, a, b)


def test_density_from_third_power(oracle_mod):
    """Section 3: the powers have no INF entry from the third one on; A and A^2 do."""
    for n in range(2, 9):
        assert (oracle_mod.power(n, 1) == INF).any()
        assert (oracle_mod.power(n, 2) == INF).any()
        assert not (oracle_mod.power(n, 3) == INF).any(), n


@pytest.mark.parametrize("n,m", [(1, m) for m in range(3, 21)] +
                         [(2, m) for m in range(3, 13)] +
                         [(3, m) for m in range(3, 11)] +
                         [(4, m) for m in range(3, 7)] +
                         [(5, 3), (5, 4), (5, 5), (6, 3), (6, 4), (7, 3)])
def test_gamma2_matches_exhaustive_search(oracle_mod, n, m):
    """Theorem 2 against exhaustive search from the definition of 2-domination."""
    assert oracle_mod.gamma2(n, m) == oracle_mod.brute_gamma2(n, m)


def test_example1_value(oracle_mod):
    """Example 1: P_4 x C_5 has a 2-dominating set of 10 vertices; none is smaller."""
    assert oracle_mod.brute_gamma2(4, 5) == 10
    assert oracle_mod.gamma2(4, 5) == 10


def test_brute_force_checker_itself(oracle_mod):
    """The exhaustive checker on sets whose status is clear by hand."""
    n, m = 2, 4
    full = (1 << (n * m)) - 1
    assert oracle_mod.brute_is_2dominating(n, m, full)
    assert not oracle_mod.brute_is_2dominating(n, m, 0)
    # one whole path row (i = 0) of P_2 x C_4: each vertex of row 1 has a
    # single S-neighbour (its own column), so this is not 2-dominating
    row0 = sum(1 << (j * n) for j in range(m))
    assert not oracle_mod.brute_is_2dominating(n, m, row0)
    # alternating checkerboard: each outside vertex sees 3 S-neighbours
    cb = sum(1 << (j * n + i) for j in range(m) for i in range(n) if (i + j) % 2 == 0)
    assert oracle_mod.brute_is_2dominating(n, m, cb)


def test_cycle_textbook(oracle_mod):
    """n = 1: gamma_2(C_m) = ceil(m/2) (textbook)."""
    g = oracle_mod.gamma2_sweep(1, 60)
    for m in range(3, 61):
        assert g[m - 1] == (m + 1) // 2


@pytest.mark.parametrize("n,mmax", [(2, 80), (3, 80), (4, 80), (5, 80), (6, 80), (7, 80), (8, 80), (9, 60)])
def test_gamma2_closed_form(oracle_mod, n, mmax):
    """Section 4 closed form with Tables 4 and 6 (and the cycle-5 exceptions)."""
    g = oracle_mod.gamma2_sweep(n, mmax)
    for m in range(3, mmax + 1):
        assert g[m - 1] == gamma2_closed_form(n, m), (n, m)


@pytest.mark.slow
def test_gamma2_closed_form_n10(oracle_mod):
    g = oracle_mod.gamma2_sweep(10, 27)
    for m in range(3, 28):
        assert g[m - 1] == gamma2_closed_form(10, m), m


def test_cycle5_column_garzon(oracle_mod):
    """gamma_2(C_5 x P_n) = 2n+2 for even n > 2, 2n+1 for n = 2 or odd n, the
    formula the paper quotes from its companion work (Section 4)."""
    for n in range(2, 9):
        expect = 2 * n + 2 if (n > 2 and n % 2 == 0) else 2 * n + 1
        assert oracle_mod.gamma2(n, 5) == expect, n


def test_multiple_of_three_statement(oracle_mod):
    """Section 4: for 8 <= n <= 12 and m = 0 (mod 3), gamma_2 = (n+2) m / 3 (n = 8 here)."""
    g = oracle_mod.gamma2_sweep(8, 48)
    for m in range(3, 49, 3):
        assert g[m - 1] == 10 * m // 3


def test_recurrence_tables_3_and_4(oracle_mod):
    """Algorithms 3 and 4 at K = 50 reproduce Tables 3 and 4 for n = 2..9."""
    t3 = {int(r[0]): tuple(int(v) for v in r[1:]) for r in read_table("table3_recurrence.txt")}
    t4 = {int(r[0]): tuple(int(v) for v in r[1:]) for r in read_table("table4_min_recurrence.txt")}
    for n in range(2, 10):
        r0, a, b, m0 = oracle_mod.recurrence(n, 50)
        assert (r0, a, b) == t3[n], n
        assert (m0, a, b) == t4[n], n


def test_lemma1_shift(oracle_mod):
    """Lemma 1: once A^(m0+a) = b (x) A^m0, every later power repeats with the same shift."""
    n, m0, a, b = 4, 9, 8, 14
    for t in range(0, 6):
        hi = oracle_mod.power(n, m0 + a + t)
        lo = oracle_mod.power(n, m0 + t)
        assert (hi == lo + b).all()
    assert not (oracle_mod.power(n, m0 - 1 + a) == oracle_mod.power(n, m0 - 1) + b).all()


def test_state_rows_are_rows_of_the_state_matrix(oracle_mod):
    """Rows built alone (the form the n = 11..13 parity tests use) equal the
    rows of the whole matrix for n = 1..9, in any order, repeated or not."""
    rng = np.random.default_rng(9)
    for n in range(1, 10):
        A = oracle_mod.state_matrix(n)
        N = A.shape[0]
        rows = np.concatenate([[0, N - 1], rng.integers(0, N, 20), [0]])
        assert (oracle_mod.state_rows(n, rows) == A[rows]).all(), n
    with pytest.raises(ValueError):
        oracle_mod.state_rows(4, [36])
    with pytest.raises(ValueError):
        oracle_mod.state_rows(4, [-1])


def test_state_rows_fixed_columns_and_rows_at_large_n(oracle_mod):
    """Two consequences of Section 2.2's rules that hold for every n, checked
    where the whole matrix is not built (n = 10..13):
    * the all-zero word can follow every word (no letter of it is 1 or 2, and
      q_i = 2 only asks p_i = 0), with label n: column 0 is n in every row;
    * after the all-2 word only the all-zero word can follow (q_i = 2 forces
      p_i = 0 at every position): that row is n at column 0 and INF elsewhere;
    * every finite entry is the number of zeros of its column's word."""
    for n in range(10, 14):
        codes = oracle_mod.words(n)
        N = codes.size
        all2 = int(np.searchsorted(codes, 3 ** n - 1))
        assert codes[all2] == 3 ** n - 1
        rows = np.array([0, 1, N // 3, N - 1, all2], dtype=np.int64)
        R = oracle_mod.state_rows(n, rows)
        assert (R[:, 0] == n).all(), n
        assert R[-1, 0] == n and (R[-1, 1:] == INF).all(), n
        fin = np.nonzero(R[:3] < INF)
        for r, c in zip(*fin):
            assert R[r, c] == oracle_mod.word_string(n, int(codes[c])).count("0")
