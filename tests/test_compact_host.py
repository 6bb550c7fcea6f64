"""The shape that compact powers rely on, on the oracle's powers of A(D_n):
from A^3 on, every entry is finite and a row's entries span at most n; under
the left step the residuals over each row's least entry never grow."""
import numpy as np
import pytest

INF = 65535


@pytest.mark.parametrize("n", range(2, 7))
def test_rows_of_powers_are_finite_and_narrow(oracle_mod, n):
    A = oracle_mod.state_matrix(n).astype(np.int64)
    P = A.copy()
    prev = None
    for k in range(2, 31):
        P = oracle_mod.minplus(A, P).astype(np.int64)
        if k < 3:
            continue
        assert (P < INF).all(), (n, k)
        lo = P.min(axis=1)
        res = P - lo[:, None]
        assert res.max() <= n, (n, k)
        if prev is not None:
            # each row's residuals are bounded by those of the successor that
            # gives its least entry, so the largest residual never grows
            assert res.max() <= prev.max(), (n, k)
        prev = res


def test_n1_keeps_infinite_entries(oracle_mod):
    """P_1 x C_m is a cycle: its powers keep INF entries (no compact form)."""
    A = oracle_mod.state_matrix(1).astype(np.int64)
    P = A.copy()
    for _ in range(2, 20):
        P = oracle_mod.minplus(A, P).astype(np.int64)
        assert (P >= INF).any()
