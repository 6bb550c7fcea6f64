// Start states pruned by the cycle's rotation symmetry.
//
// A closed walk of length m in D_n visits m states, and its label (the size
// of the 2-dominating set it encodes, Theorem 2) is the sum of their zero
// counts.  The state with the fewest zeros on an optimal walk therefore has
// at most floor(gamma_2 / m) zeros, and the walk may start there (rotating
// the cycle).  So gamma_2 = min over the states i with at most
// floor(gamma_2 / m) zeros of (A^m)_ii, and only those columns of the powers
// are needed: A^m e_i for i in S, a chain on an N x |S| panel.
//
// Kernels: the columns S of A(D_n) as a dense panel, and the minimum of the
// selected diagonal entries X[S[j]][j] of a panel.
#include "device_core.hpp"

namespace tp {

namespace {

// block (q, y): X[q][j] = A[q][idx[j]] for j in [1024 y, 1024 (y + 1)); an
// index outside 0..N-1 gives an INF column
__global__ void state_columns_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                     const int32_t *__restrict__ idx, int64_t count,
                                     uint16_t *__restrict__ X, int64_t ldx) {
  const int64_t q = blockIdx.x;
  const uint32_t mq = masks[q];
  uint16_t *row = X + q * ldx;
  const int64_t j0 = (int64_t)blockIdx.y * blockDim.x * 4;
  for (int t = 0; t < 4; ++t) {
    const int64_t j = j0 + (int64_t)t * blockDim.x + threadIdx.x;
    if (j >= count) break;
    const int64_t p = idx[j];
    if (p < 0 || p >= N) {
      row[j] = kInf16;
      continue;
    }
    const uint32_t mp = masks[p];
    row[j] = can_follow(mq, mp, full) ? (uint16_t)__builtin_popcount(mp & 0xFFFFu) : kInf16;
  }
}

// out[0] = min_j X[idx[j]][j] over the indices inside 0..rows-1 (INF when
// none); one block
__global__ void __launch_bounds__(1024) diag_select_kernel(int64_t rows, int64_t count,
                                                           const int32_t *__restrict__ idx,
                                                           const uint16_t *__restrict__ X,
                                                           int64_t ldx, int32_t *__restrict__ out) {
  __shared__ int32_t red[16];
  int32_t best = kInf16;
  for (int64_t j = threadIdx.x; j < count; j += blockDim.x) {
    const int64_t r = idx[j];
    if (r >= 0 && r < rows) best = min(best, (int32_t)X[r * ldx + j]);
  }
  for (int o = 32; o >= 1; o >>= 1) best = min(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = min(r, red[w]);
    out[0] = r;
  }
}

}  // namespace

hipError_t launch_state_columns(int n, int64_t N, const uint32_t *masks, const int32_t *idx,
                                int64_t count, uint16_t *X, int64_t ldx, hipStream_t s) {
  if (N == 0 || count == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int bs = 256;
  const dim3 grid((unsigned)N, (unsigned)((count + bs * 4 - 1) / (bs * 4)));
  hipLaunchKernelGGL(state_columns_kernel, grid, dim3(bs), 0, s, N, full, masks, idx, count, X,
                     ldx);
  return hipGetLastError();
}

hipError_t launch_diag_select_min(int64_t rows, int64_t count, const int32_t *idx,
                                  const uint16_t *X, int64_t ldx, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(diag_select_kernel, dim3(1), dim3(1024), 0, s, rows, count, idx, X, ldx,
                     out);
  return hipGetLastError();
}

}  // namespace tp
