"""tp_minplus_gemm_ex_noalloc, the split-K product for callers that cannot
allocate, against tp_minplus_gemm_ex (the same product with library-owned
scratch) through the C ABI: two calls in a row, the second on a smaller
input, bit-exact, with and without accumulation; a product whose partials
exceed the fixed buffer is refused and leaves C as it was."""
import sys

import numpy as np
import pytest

import synth

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


def dev16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint16).view(np.int16)).cuda() \
        .view(torch.uint16)


def host16(t):
    import torch
    torch.cuda.synchronize()
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


def call(fn, A, B, C, acc, config, ksplit):
    M, K = A.shape
    N = B.shape[1]
    return fn(2, M, N, K, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), C.data_ptr(),
              C.stride(0), acc, config, ksplit, None)


def test_noalloc_matches_gemm_ex_twice_then_smaller(tp):
    import torch
    cases = [(1386, 1386, 1386, 0, 8), (300, 517, 2000, 3, 4)]  # second call smaller
    for i, (M, N, K, config, ksplit) in enumerate(cases):
        say("no-alloc product", M, N, K, config, ksplit)
        A = dev16(synth.stress_matrix(M, K, 10 + i, 0, 30000, 0.3, np.uint16))
        B = dev16(synth.stress_matrix(K, N, 20 + i, 0, 30000, 0.3, np.uint16))
        C0 = dev16(synth.stress_matrix(M, N, 30 + i, 0, 60000, 0.1, np.uint16))
        for acc in (0, 1):
            ref = C0.clone()
            got = C0.clone()
            assert call(tp.lib.tp_minplus_gemm_ex, A, B, ref, acc, config, ksplit) == 0
            assert call(tp.lib.tp_minplus_gemm_ex_noalloc, A, B, got, acc, config, ksplit) == 0
            assert np.array_equal(host16(got), host16(ref)), (M, N, K, acc)


def test_noalloc_refuses_oversized_partials(tp):
    import torch
    say("no-alloc refusal")
    M = N = K = 4096  # 4 slices of 4096 x 4096 u16 partials: 128 MiB > 64 MiB
    A = torch.zeros((M, K), dtype=torch.uint16, device="cuda")
    B = torch.zeros((K, N), dtype=torch.uint16, device="cuda")
    C = torch.full((M, N), 7, dtype=torch.uint16, device="cuda")
    assert call(tp.lib.tp_minplus_gemm_ex_noalloc, A, B, C, 0, 0, 4) == tp.TP_EINVAL
    assert "scratch" in tp.lib.tp_last_error().decode()
    torch.cuda.synchronize()
    assert bool((C == 7).all())
    # the same product unsplit needs no scratch and runs
    assert call(tp.lib.tp_minplus_gemm_ex_noalloc, A, B, C, 0, 0, 1) == 0
    torch.cuda.synchronize()
    assert bool((C == 0).all())
