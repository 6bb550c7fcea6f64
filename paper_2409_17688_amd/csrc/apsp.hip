// All-pairs shortest paths by (min,+) squaring: the same semiring and the
// same dense product as the powers of A(D_n).
//
// With non-negative integer weights W (INF = no arc) and I the (min,+)
// identity (0 on the diagonal, INF elsewhere), (I + W)^k holds the least
// weight of a path of at most k arcs, so after t = ceil(log2(N - 1))
// squarings every shortest path (at most N - 1 arcs) is covered.  Sums
// saturate at INF in every step; as all weights are non-negative, a path's
// saturated sum is min(its weight, INF) whatever the order of the additions,
// so each entry is exactly min(distance, INF).
#include <algorithm>
#include <utility>

#include "device_core.hpp"

namespace tp {

namespace {

// D[i][j] = (i == j) ? 0 : W[i][j]: the identity taken in, i.e. min(W, I)
// for non-negative W.  D may be W itself.
// Block (i, y) covers row i, columns y * 256 + 256 * gridDim.y * r.
template <typename T>
__global__ void closure_start_kernel(int64_t N, const T *W, int64_t ldw, T *D, int64_t ldd) {
  const int64_t i = blockIdx.x;
  for (int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; j < N;
       j += (int64_t)gridDim.y * blockDim.x)
    D[i * ldd + j] = (i == j) ? (T)0 : W[i * ldw + j];
}

int squarings(int64_t N) {
  int t = 0;
  while (((int64_t)1 << t) < N - 1) ++t;
  return t;
}

}  // namespace

}  // namespace tp

using namespace tp;

extern "C" {

int tp_apsp(int dtype, int64_t N, const void *d_W, int64_t ldw, void *d_D, int64_t ldd,
            void *d_T, int64_t ldt, hipStream_t stream) {
  TP_REQUIRE(dtype == TP_U8 || dtype == TP_U16, "bad dtype %d", dtype);
  TP_REQUIRE(N >= 0 && N < ((int64_t)1 << 31), "N out of range");
  if (N == 0) return TP_OK;
  TP_REQUIRE(d_W != nullptr && d_D != nullptr, "NULL matrix");
  TP_REQUIRE(ldw >= N && ldd >= N, "leading dimension below N");
  const int t = squarings(N);
  TP_REQUIRE(t == 0 || (d_T != nullptr && ldt >= N && d_T != d_D && d_T != d_W),
             "the work matrix T must be N x N and distinct from D and W");
  // start in T when the number of squarings is odd, so the last lands in D
  void *cur = (t % 2 == 1) ? d_T : d_D;
  void *oth = (t % 2 == 1) ? d_D : d_T;
  int64_t ldc = (t % 2 == 1) ? ldt : ldd, ldo = (t % 2 == 1) ? ldd : ldt;
  const dim3 grid((unsigned)N, (unsigned)std::min<int64_t>((N + 255) / 256, 64));
  if (dtype == TP_U16)
    hipLaunchKernelGGL(closure_start_kernel<uint16_t>, grid, dim3(256), 0, stream, N,
                       (const uint16_t *)d_W, ldw, (uint16_t *)cur, ldc);
  else
    hipLaunchKernelGGL(closure_start_kernel<uint8_t>, grid, dim3(256), 0, stream, N,
                       (const uint8_t *)d_W, ldw, (uint8_t *)cur, ldc);
  TP_HIP_CHECK(hipGetLastError());
  for (int s = 0; s < t; ++s) {
    TP_HIP_CHECK(launch_gemm(dtype, N, N, N, cur, ldc, cur, ldc, oth, ldo, 0, -1, 0, stream));
    std::swap(cur, oth);
    std::swap(ldc, ldo);
  }
  return TP_OK;
}

}  // extern "C"
