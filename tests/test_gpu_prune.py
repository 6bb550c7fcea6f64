"""Start-state pruning by the cycle's rotation symmetry: the state selection,
the column panel of A(D_n) and the selected-diagonal minimum against the
oracle, and the plain path with pruning forced against the oracle and the
closed form."""
import numpy as np
import pytest

from closed_form import gamma2_closed_form

pytestmark = pytest.mark.gpu

INF = 65535


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_17688_amd as tp
    return tp


def _zeros(oracle_mod, n):
    return np.array([oracle_mod.zeros(n, int(c)) for c in oracle_mod.words(n)])


@pytest.mark.parametrize("n", range(1, 10))
def test_state_select_matches_oracle(tp, oracle_mod, n):
    z = _zeros(oracle_mod, n)
    for k in range(0, n + 2):
        got = tp.tp_state_select(n, k).cpu().numpy()
        assert list(got) == list(np.nonzero(z <= k)[0]), (n, k)


@pytest.mark.parametrize("n", [2, 5, 7, 8])
def test_state_columns_match_oracle(tp, oracle_mod, n):
    import torch
    A = oracle_mod.state_matrix(n)
    N = A.shape[0]
    rng = np.random.default_rng(n)
    idx = rng.integers(0, N, size=min(N, 300)).astype(np.int32)
    idx[::7] = -1  # out of range: INF columns
    idx[3::11] = N + 5
    X = tp.tp_build_state_columns(n, torch.from_numpy(idx).cuda()).cpu().numpy().astype(np.int64)
    for j, p in enumerate(idx):
        want = A[:, p] if 0 <= p < N else np.full(N, INF)
        assert (X[:, j] == want).all(), (n, j, p)


def test_diag_select_min_matches_definition(tp):
    import torch
    rng = np.random.default_rng(3)
    for rows, cnt in ((1, 1), (37, 20), (500, 333), (2000, 1500)):
        M = rng.integers(0, INF + 1, size=(rows, cnt)).astype(np.uint16)
        idx = rng.integers(-3, rows + 3, size=cnt).astype(np.int32)
        Xd = torch.from_numpy(M.view(np.int16)).cuda().view(torch.uint16)
        got = int(tp.tp_diag_select_min(Xd, torch.from_numpy(idx).cuda()).item())
        vals = [int(M[r, j]) for j, r in enumerate(idx) if 0 <= r < rows]
        assert got == (min(vals) if vals else INF), (rows, cnt)


def test_pruned_chain_from_the_pieces(tp, oracle_mod):
    """gamma_2 = min over the states with at most floor(gamma_2 / m) zeros of
    (A^m)_ii, with the library's pieces: selection, column panel, sparse left
    steps on the panel, selected diagonal."""
    import torch
    for n in (3, 6, 8):
        g = oracle_mod.gamma2_sweep(n, 40)
        for m in (3, 4, 5, 11, 24, 40):
            k = int(g[m - 1]) // m
            idx = tp.tp_state_select(n, k)
            X = tp.tp_build_state_columns(n, idx)
            for _ in range(m - 1):
                Y = torch.empty_like(X)
                X = tp.tp_state_left_mul(n, X, Y)
            assert int(tp.tp_diag_select_min(X, idx).item()) == g[m - 1], (n, m)


@pytest.fixture
def forced(tp):
    tp.tp_tune_prune(1)
    yield
    tp.tp_tune_prune(0)


def test_plain_path_pruned_matches_oracle(tp, oracle_mod, forced):
    for n in range(1, 9):
        g = oracle_mod.gamma2_sweep(n, 60)
        for m in range(3, 61):
            assert tp.tp_tropical_power_trace(n, m) == g[m - 1], (n, m)


@pytest.mark.parametrize("n,ms", [(9, [3, 4, 5, 17, 100]), (10, [3, 4, 5, 31, 64]),
                                  (11, [3, 4, 5, 22]), (12, [3, 4, 5, 7, 30])])
def test_plain_path_pruned_matches_closed_form(tp, forced, n, ms):
    # m = 4 at n = 12 needs the second pass (gamma_2 = 20 = 5 m)
    for m in ms:
        assert tp.tp_tropical_power_trace(n, m) == gamma2_closed_form(n, m), (n, m)


def test_prune_mode_rejects_bad_values(tp):
    with pytest.raises(tp.TropicalError):
        tp.tp_tune_prune(2)
    with pytest.raises(tp.TropicalError):
        tp.tp_state_select(0, 1)


def test_pruned_compact_chain_matches_oracle_and_16_bits(tp, oracle_mod, forced):
    """The pruned plain path with its chain on shared-base compact powers
    (forced from n = 2 on; n = 1 never holds and falls back): the oracle's
    gamma_2 for n <= 8, m <= 40, and the 16-bit chain's for n = 9, 10."""
    try:
        tp.tp_tune_compact_chains(2)
        for n in range(1, 9):
            g = oracle_mod.gamma2_sweep(n, 40)
            for m in range(3, 41):
                assert tp.tp_tropical_power_trace(n, m) == g[m - 1], (n, m)
        got = {(n, m): tp.tp_tropical_power_trace(n, m) for n in (9, 10) for m in (5, 6, 13, 40)}
        tp.tp_tune_compact_chains(0)
        for (n, m), v in got.items():
            assert v == tp.tp_tropical_power_trace(n, m) == gamma2_closed_form(n, m), (n, m)
    finally:
        tp.tp_tune_compact_chains(11)
