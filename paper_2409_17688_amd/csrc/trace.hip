// Traces (Theorem 2: gamma_2 is the minimum of the diagonal of A(D_n)^m,
// Algorithm 5 reads it off every power).
//
//   trace_min          min_i X_ii                     reads N entries
//   trace_of_product   min_i (X x Y)_ii = min_{i,k} x_ik + y_ki
//                                                     reads 2 N^2 entries
// The second one closes a power chain without forming its last product: with
// X = A^a and Y = A^b it gives gamma_2 for m = a + b at the price of one pass
// over two matrices, which is bound by HBM bandwidth.  Both matrices stream
// row-wise in 16-byte loads; Y's 8 x 8 blocks are transposed in registers.
#include <algorithm>

#include "device_core.hpp"

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

// Waves walk 64 x 64 tiles (i-block, k-block) with a grid stride, each tile
// by one wave with its Y block transposed in registers (trace_tile_regs);
// the partial minimum is folded into *out with one atomic per workgroup.
template <typename T, bool VEC>
__global__ void __launch_bounds__(256) trace_of_product_kernel(int64_t N, const T *__restrict__ X,
                                                               int64_t ldx,
                                                               const T *__restrict__ Y,
                                                               int64_t ldy, int64_t tiles,
                                                               int32_t *__restrict__ out) {
  __shared__ int32_t part[4];
  u16x2 acc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = splat(0xFFFFu);
  const int lane = threadIdx.x & 63;
  const int64_t wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t total = tiles * tiles;
  for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < total; t += (int64_t)gridDim.x * 4)
    trace_tile_regs<T, VEC>(X, ldx, Y, ldy, N, (t % tiles) * 64, (t / tiles) * 64, lane, acc);
  const int32_t best = min(block_min(acc, part), inf_of<T>());
  if (threadIdx.x == 0 && best < inf_of<T>()) atomicMin(out, best);
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
  const int64_t tiles = (N + 63) / 64;
  const int64_t blocks = std::min<int64_t>((tiles * tiles + 3) / 4, 2048);  // a tile per wave
  const int64_t VE = 8;
  const size_t es = dtype == TP_U16 ? 2 : 1;
  const bool vec = (ldx % VE == 0) && (ldy % VE == 0) && ((uintptr_t)X % (VE * es) == 0) &&
                   ((uintptr_t)Y % (VE * es) == 0);
#define TP_TRACE_LAUNCH(T, V)                                                                  \
  hipLaunchKernelGGL((trace_of_product_kernel<T, V>), dim3((unsigned)blocks), dim3(256), 0, s, \
                     N, (const T *)X, ldx, (const T *)Y, ldy, tiles, out)
  if (dtype == TP_U16) {
    if (vec) TP_TRACE_LAUNCH(uint16_t, true);
    else TP_TRACE_LAUNCH(uint16_t, false);
  } else {
    if (vec) TP_TRACE_LAUNCH(uint8_t, true);
    else TP_TRACE_LAUNCH(uint8_t, false);
  }
#undef TP_TRACE_LAUNCH
  return hipGetLastError();
}

}  // namespace tp
