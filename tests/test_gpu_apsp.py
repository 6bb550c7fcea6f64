"""All-pairs shortest paths by (min,+) squaring against the oracle's
Floyd-Warshall relaxation."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_17688_amd as tp
    return tp


def _dev(torch, M, dtype, ld=None):
    N = M.shape[0]
    ld = ld or max(N, 1)
    np_t = np.uint16 if dtype == "u16" else np.uint8
    buf = np.full((N, ld), 7, dtype=np_t)
    buf[:, :N] = M.astype(np_t)
    if dtype == "u16":
        t = torch.from_numpy(buf.view(np.int16)).cuda().view(torch.uint16)
    else:
        t = torch.from_numpy(buf).cuda()
    return t[:, :N]


def _graph(seed, N, p, hi, inf):
    rng = np.random.default_rng(seed)
    W = rng.integers(0, hi, (N, N))
    W[rng.random((N, N)) > p] = inf
    return W


@pytest.mark.parametrize("N", [1, 2, 3, 5, 37, 130, 600, 1100])
def test_apsp_u16_matches_oracle(tp, oracle_mod, N):
    import torch
    W = _graph(N, N, 0.05 if N > 100 else 0.3, 50, 65535)
    ld = (N + 63) // 64 * 64
    D = tp.tp_apsp(_dev(torch, W, "u16", ld), _dev(torch, np.zeros((N, N)), "u16", ld),
                   _dev(torch, np.zeros((N, N)), "u16", ld))
    got = D.cpu().numpy().astype(np.int64)
    assert (got == oracle_mod.apsp(W, 65535)).all(), N


@pytest.mark.parametrize("N", [3, 64, 129])
def test_apsp_u8_matches_oracle(tp, oracle_mod, N):
    import torch
    W = _graph(100 + N, N, 0.08, 4, 255)
    D = tp.tp_apsp(_dev(torch, W, "u8"))
    assert (D.cpu().numpy().astype(np.int64) == oracle_mod.apsp(W, 255)).all(), N


def test_apsp_saturates_like_the_oracle(tp, oracle_mod):
    import torch
    W = _graph(7, 200, 0.1, 30000, 65535)
    W[W < 65535] += 20000  # paths of three or more arcs saturate
    D = tp.tp_apsp(_dev(torch, W, "u16"))
    assert (D.cpu().numpy().astype(np.int64) == oracle_mod.apsp(W, 65535)).all()


def test_apsp_in_place(tp, oracle_mod):
    import torch
    W = _graph(9, 300, 0.02, 50, 65535)
    Wd = _dev(torch, W, "u16")
    T = torch.empty_like(Wd)
    D = tp.tp_apsp(Wd, Wd, T)
    assert D.data_ptr() == Wd.data_ptr()
    assert (D.cpu().numpy().astype(np.int64) == oracle_mod.apsp(W, 65535)).all()


def test_apsp_rejects_bad_arguments(tp):
    import torch
    W = torch.zeros((8, 8), dtype=torch.uint16, device="cuda")
    with pytest.raises(tp.TropicalError):
        tp.tp_apsp(W, W, W)  # T is W
    D = torch.zeros_like(W)
    with pytest.raises(tp.TropicalError):
        tp.tp_apsp(W, D, D)  # T is D
    lib = tp.lib
    assert lib.tp_apsp(3, 8, W.data_ptr(), 8, D.data_ptr(), 8, None, 8, None) == tp.TP_EINVAL
    assert lib.tp_apsp(2, 8, W.data_ptr(), 8, D.data_ptr(), 8, None, 8, None) == tp.TP_EINVAL
