"""Algorithm 3's constant-difference test in the oracle, pinned by hand-made
cases, and the library's host-side solution of Theorem 3's finite difference
equation fed with the oracle's recurrence (no GPU work)."""
import numpy as np
import pytest

from closed_form import gamma2_closed_form
from conftest import read_table

INF = 65535


def test_constant_difference_cases(oracle_mod):
    rng = np.random.default_rng(5)
    Y = rng.integers(0, 200, (9, 9)).astype(np.int32)
    Y[rng.random((9, 9)) < 0.3] = INF
    X = np.where(Y >= INF, INF, Y + 3)
    assert oracle_mod.constant_difference(X, Y) == (True, 3)
    assert oracle_mod.constant_difference(Y, Y) == (True, 0)
    # a negative constant is a constant too
    assert oracle_mod.constant_difference(Y, X) == (True, -3)
    bad = X.copy()
    i, j = np.argwhere(Y < INF)[4]
    bad[i, j] += 1
    assert oracle_mod.constant_difference(bad, Y)[0] is False
    # an INF pattern that differs fails whatever the finite entries do
    bad = X.copy()
    bad[i, j] = INF
    assert oracle_mod.constant_difference(bad, Y)[0] is False
    # no finite entry: holds with b = 0
    full = np.full((4, 4), INF, np.int32)
    assert oracle_mod.constant_difference(full, full) == (True, 0)


def test_recurrence_on_the_shifted_powers(oracle_mod):
    """Table 3 row n = 4 (r0 = 42, a = 8, b = 14) seen directly on the powers."""
    hi, lo = oracle_mod.power(4, 50), oracle_mod.power(4, 42)
    assert oracle_mod.constant_difference(hi, lo) == (True, 14)
    assert oracle_mod.constant_difference(hi, oracle_mod.power(4, 43))[0] is False


@pytest.fixture(scope="module")
def tp():
    import paper_2409_17688_amd as tp
    return tp


def _rec_from_oracle(tp, oracle_mod, n, K):
    got = oracle_mod.recurrence(n, K)
    rec = tp.Recurrence()
    rec.K, rec.window = K, K - 1
    if got is not None:
        rec.found = 1
        rec.r0, rec.a, rec.b, rec.n0 = got
    return rec, oracle_mod.gamma2_sweep(n, K)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_theorem3_solution_matches_closed_form(tp, oracle_mod, n):
    rec, diag = _rec_from_oracle(tp, oracle_mod, n, 50)
    assert rec.found
    for m in range(3, 600):
        assert tp.tp_gamma2_recurrence(rec, diag, m) == gamma2_closed_form(n, m), (n, m)


@pytest.mark.parametrize("n", [3, 5, 6])
def test_theorem3_solution_matches_the_chain(tp, oracle_mod, n):
    rec, diag = _rec_from_oracle(tp, oracle_mod, n, 50)
    long = oracle_mod.gamma2_sweep(n, 300)
    for m in range(3, 301):
        assert tp.tp_gamma2_recurrence(rec, diag, m) == long[m - 1], (n, m)


def test_theorem3_rejects_what_it_cannot_answer(tp, oracle_mod):
    rec, diag = _rec_from_oracle(tp, oracle_mod, 8, 12)
    # n = 8 repeats only from its 25th power on (Table 4): not within 12
    t4 = {int(r[0]): int(r[1]) for r in read_table("table4_min_recurrence.txt")}
    assert t4[8] > 12
    assert tp.tp_gamma2_recurrence(rec, diag, 12) == diag[11]
    with pytest.raises(tp.TropicalError):
        tp.tp_gamma2_recurrence(rec, diag, 13)
    with pytest.raises(tp.TropicalError):
        tp.tp_gamma2_recurrence(rec, diag, 2)
    with pytest.raises(ValueError):
        tp.tp_gamma2_recurrence(rec, diag[:5], 4)


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_rotation_pruning_on_the_oracle(oracle_mod, n):
    """A closed walk's label is the sum of the zero counts of the m states it
    visits, so an optimal one passes through a state with at most
    floor(gamma_2 / m) zeros: the minimum over those diagonal entries alone
    is gamma_2 (checked on the oracle's powers)."""
    z = np.array([oracle_mod.zeros(n, int(c)) for c in oracle_mod.words(n)])
    for m in range(3, 16):
        P = oracle_mod.power(n, m)
        g = int(P.diagonal().min())
        k = g // m
        assert int(P.diagonal()[z <= k].min()) == g, (n, m)
