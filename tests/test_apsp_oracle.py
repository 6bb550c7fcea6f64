"""The oracle's all-pairs shortest paths (Floyd-Warshall relaxation) pinned
to hand-worked graphs and to Dijkstra's algorithm run from every vertex."""
import numpy as np
import pytest

INF = 65535


def test_hand_worked_graphs(oracle_mod):
    # 0 -> 1 (3), 1 -> 2 (4), 0 -> 2 (9), 2 -> 0 (1); vertex 3 isolated
    W = np.full((4, 4), INF)
    W[0, 1], W[1, 2], W[0, 2], W[2, 0] = 3, 4, 9, 1
    D = oracle_mod.apsp(W)
    want = np.array([[0, 3, 7, INF], [5, 0, 4, INF], [1, 4, 0, INF], [INF, INF, INF, 0]])
    assert (D == want).all()
    # sums saturate at INF
    W = np.full((3, 3), INF)
    W[0, 1], W[1, 2] = 40000, 40000
    D = oracle_mod.apsp(W)
    assert D[0, 2] == INF and D[0, 1] == 40000


def _dijkstra(W, s):
    """Textbook Dijkstra from s (non-negative weights), distances capped at INF."""
    import heapq
    N = W.shape[0]
    d = [None] * N
    d[s] = 0
    heap = [(0, s)]
    done = [False] * N
    while heap:
        du, u = heapq.heappop(heap)
        if done[u]:
            continue
        done[u] = True
        for v in range(N):
            w = int(W[u, v])
            if w < INF and (d[v] is None or du + w < d[v]):
                d[v] = du + w
                heapq.heappush(heap, (d[v], v))
    return [INF if x is None else min(x, INF) for x in d]


@pytest.mark.parametrize("seed,N,p", [(0, 30, 0.2), (1, 60, 0.05), (2, 120, 0.5), (3, 1, 0.5),
                                      (4, 25, 0.3)])
def test_matches_dijkstra(oracle_mod, seed, N, p):
    rng = np.random.default_rng(seed)
    W = rng.integers(0, 50, (N, N))
    W[rng.random((N, N)) > p] = INF
    if seed == 4:
        W[W < INF] += 30000  # two arcs already saturate
    D = oracle_mod.apsp(W)
    for s in range(N):
        assert list(D[s]) == _dijkstra(W, s), (seed, s)
