// Traces (Theorem 2: gamma_2 is the minimum of the diagonal of A(D_n)^m,
// Algorithm 5 reads it off every power).
//
//   trace_min          min_i X_ii                     reads N entries
//   trace_of_product   min_i (X x Y)_ii = min_{i,k} x_ik + y_ki
//                                                     reads 2 N^2 entries
// The second one closes a power chain without forming its last product: with
// X = A^a and Y = A^b it gives gamma_2 for m = a + b at the price of one pass
// over two matrices, which is bound by HBM bandwidth.  Y is read in 64 x 64
// tiles through LDS so that both matrices stream row-wise.
#include "common.hpp"

namespace tp {

namespace {

template <typename T>
constexpr int32_t inf_of() {
  return sizeof(T) == 2 ? 0xFFFF : 0xFF;
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

__global__ void fill_bytes_kernel(uint8_t *p, size_t count, uint8_t value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

template <typename T>
__global__ void __launch_bounds__(1024) trace_min_kernel(int64_t N, const T *__restrict__ X,
                                                         int64_t ldx, int32_t *__restrict__ out) {
  __shared__ int32_t part[16];
  int32_t best = inf_of<T>();
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) best = min(best, (int32_t)X[i * ldx + i]);
  for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = min(best, part[w]);
    *out = best;
  }
}

// One workgroup per 64 x 64 tile (i-block, k-block): every x_ik + y_ki of the
// tile, reduced and folded into *out with an atomic min.
template <typename T>
__global__ void __launch_bounds__(256) trace_of_product_kernel(int64_t N, const T *__restrict__ X,
                                                               int64_t ldx,
                                                               const T *__restrict__ Y,
                                                               int64_t ldy, int tiles,
                                                               int32_t *__restrict__ out) {
  __shared__ uint16_t yt[64][65];  // yt[i][k] = Y[k0 + k][i0 + i]
  __shared__ int32_t part[4];
  const int tid = threadIdx.x;
  const int ti = blockIdx.x % tiles, tk = blockIdx.x / tiles;
  const int64_t i0 = (int64_t)ti * 64, k0 = (int64_t)tk * 64;
  const int32_t inf = inf_of<T>();
  // stage Y[k0..k0+63][i0..i0+63] transposed: thread reads row k, 16 columns
  {
    const int kr = tid >> 2, ic = (tid & 3) * 16;
    const int64_t k = k0 + kr;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t i = i0 + ic + e;
      yt[ic + e][kr] = (k < N && i < N) ? (uint16_t)Y[k * ldy + i] : (uint16_t)inf;
    }
  }
  __syncthreads();
  // each thread: row i = i0 + tid / 4, 16 consecutive k
  int32_t best = inf;
  {
    const int ir = tid >> 2, kc = (tid & 3) * 16;
    const int64_t i = i0 + ir;
    if (i < N) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t k = k0 + kc + e;
        if (k < N) best = min(best, (int32_t)X[i * ldx + k] + (int32_t)yt[ir][kc + e]);
      }
    }
  }
  best = min(best, inf);
  for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
  if ((tid & 63) == 0) part[tid >> 6] = best;
  __syncthreads();
  if (tid == 0) {
    best = min(min(part[0], part[1]), min(part[2], part[3]));
    if (best < inf) atomicMin(out, best);
  }
}

}  // namespace

hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                     count, value);
  return hipGetLastError();
}

hipError_t launch_fill_bytes(void *p, size_t count, uint8_t value, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_bytes_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     (uint8_t *)p, count, value);
  return hipGetLastError();
}

hipError_t launch_trace_min(int dtype, int64_t N, const void *X, int64_t ldx, int32_t *out,
                            hipStream_t s) {
  if (dtype == TP_U16)
    hipLaunchKernelGGL(trace_min_kernel<uint16_t>, dim3(1), dim3(1024), 0, s, N,
                       (const uint16_t *)X, ldx, out);
  else
    hipLaunchKernelGGL(trace_min_kernel<uint8_t>, dim3(1), dim3(1024), 0, s, N,
                       (const uint8_t *)X, ldx, out);
  return hipGetLastError();
}

hipError_t launch_trace_of_product(int dtype, int64_t N, const void *X, int64_t ldx,
                                   const void *Y, int64_t ldy, int32_t *out, hipStream_t s) {
  hipError_t e = launch_fill_i32(out, 1, dtype == TP_U16 ? 0xFFFF : 0xFF, s);
  if (e != hipSuccess || N == 0) return e;
  const int tiles = (int)((N + 63) / 64);
  const int64_t blocks = (int64_t)tiles * tiles;
  if (dtype == TP_U16)
    hipLaunchKernelGGL(trace_of_product_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       N, (const uint16_t *)X, ldx, (const uint16_t *)Y, ldy, tiles, out);
  else
    hipLaunchKernelGGL(trace_of_product_kernel<uint8_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       N, (const uint8_t *)X, ldx, (const uint8_t *)Y, ldy, tiles, out);
  return hipGetLastError();
}

}  // namespace tp
