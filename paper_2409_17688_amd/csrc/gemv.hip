// (min,+) matrix-vector products (Section 1 semiring; the complementary
// problem of small cycles is solved with these in the paper's companion
// work):
//   trans = 0:  y_i = min_k a_ik + x_k   (one wave per row, lanes stride k)
//   trans = 1:  y_k = min_i x_i + a_ik   (lanes own 2 columns, 16 waves split
//                                         the rows and meet in LDS)
// Both read the matrix once and are bound by HBM bandwidth.
#include "common.hpp"

namespace tp {

namespace {

template <typename T>
constexpr uint16_t inf_of() {
  return sizeof(T) == 2 ? 0xFFFFu : 0xFFu;
}

template <typename T>
__global__ void __launch_bounds__(256) gemv_rows_kernel(int64_t M, int64_t K,
                                                        const T *__restrict__ A, int64_t lda,
                                                        const T *__restrict__ x,
                                                        T *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;
  const T *row = A + i * lda;
  uint32_t best = 0xFFFFu;
  for (int64_t k = lane; k < K; k += 64) {
    const uint32_t s = (uint32_t)row[k] + (uint32_t)x[k];
    best = min(best, s);
  }
  for (int off = 32; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off));
  if (lane == 0) y[i] = (T)min(best, (uint32_t)inf_of<T>());
}

// 1024 lanes per workgroup: 16 waves split the rows, each lane owns two
// adjacent columns; the 16 partial minima meet in LDS and one lane per column
// pair writes the result.  128 columns per workgroup.
template <typename T>
__global__ void __launch_bounds__(1024) gemv_cols_kernel(int64_t M, int64_t K,
                                                         const T *__restrict__ A, int64_t lda,
                                                         const T *__restrict__ x,
                                                         T *__restrict__ y) {
  __shared__ uint32_t part[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = ((int64_t)blockIdx.x * 64 + lane) * 2;
  const bool have0 = c < K, have1 = c + 1 < K;
  u16x2 acc = splat(0xFFFFu);
  if (have0) {
    for (int64_t r = wave; r < M; r += 16) {
      const uint16_t xr = x[r];
      const uint16_t a0 = A[r * lda + c];
      const uint16_t a1 = have1 ? (uint16_t)A[r * lda + c + 1] : (uint16_t)0xFFFFu;
      acc = pk_min(acc, pk_add_sat(splat(xr), u16x2{a0, a1}));
    }
  }
  part[wave][lane] = as_u32(acc);
  __syncthreads();
  if (wave == 0 && have0) {
    for (int w = 1; w < 16; ++w) acc = pk_min(acc, as_pk(part[w][lane]));
    y[c] = (T)min((uint32_t)acc.x, (uint32_t)inf_of<T>());
    if (have1) y[c + 1] = (T)min((uint32_t)acc.y, (uint32_t)inf_of<T>());
  }
}

}  // namespace

hipError_t launch_gemv(int dtype, int64_t M, int64_t K, const void *A, int64_t lda,
                       const void *x, void *y, int trans, hipStream_t s) {
  if (!trans) {
    if (M == 0) return hipSuccess;
    dim3 grid((unsigned)((M + 3) / 4));
    if (dtype == TP_U16)
      hipLaunchKernelGGL(gemv_rows_kernel<uint16_t>, grid, dim3(256), 0, s, M, K,
                         (const uint16_t *)A, lda, (const uint16_t *)x, (uint16_t *)y);
    else
      hipLaunchKernelGGL(gemv_rows_kernel<uint8_t>, grid, dim3(256), 0, s, M, K,
                         (const uint8_t *)A, lda, (const uint8_t *)x, (uint8_t *)y);
    return hipGetLastError();
  }
  if (K == 0) return hipSuccess;
  dim3 grid((unsigned)((K + 127) / 128));
  if (dtype == TP_U16)
    hipLaunchKernelGGL(gemv_cols_kernel<uint16_t>, grid, dim3(1024), 0, s, M, K,
                       (const uint16_t *)A, lda, (const uint16_t *)x, (uint16_t *)y);
  else
    hipLaunchKernelGGL(gemv_cols_kernel<uint8_t>, grid, dim3(1024), 0, s, M, K,
                       (const uint8_t *)A, lda, (const uint8_t *)x, (uint8_t *)y);
  return hipGetLastError();
}

}  // namespace tp
