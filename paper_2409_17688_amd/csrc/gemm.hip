// Dense (min,+) matrix product C = A x B (Section 1: (A x B)_ij =
// min_k a_ik + b_kj), the product Algorithm 2 repeats for every power.
//
// The tile arithmetic lives in gemm_core.hpp.  This file launches one
// workgroup per tile, numbered so that each XCD (the hardware deals
// workgroups to the 8 XCDs in turn) gets a contiguous range of tiles, walked
// in groups of 8 tile rows, to keep A and B slabs shared in that XCD's L2.
#include "gemm_core.hpp"

namespace tp {

namespace {

constexpr int kThreads = kGemmThreads;
constexpr int kGroupM = 8;

// Maps the hardware workgroup id to a tile id such that each of the 8 XCDs
// receives a contiguous range of tiles (a bijection on [0, num_tiles)).
__device__ __forceinline__ int xcd_tile(int bid, int num_tiles) {
  const int q = num_tiles >> 3, r = num_tiles & 7;
  const int x = bid & 7, local = bid >> 3;
  return x * q + min(x, r) + local;
}

template <int BM, int BN, int BK, int TM, int TN, int MINB, typename T, bool VEC>
__global__ void __launch_bounds__(kThreads, MINB)
    minplus_gemm_kernel(int M, int N, int K, const T *__restrict__ A, int64_t lda,
                        const T *__restrict__ B, int64_t ldb, T *__restrict__ C, int64_t ldc,
                        int accumulate, int tiles_m, int tiles_n) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BK][BM];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BK][BN];
  const int num_tiles = tiles_m * tiles_n;
  const int t = xcd_tile(blockIdx.x, num_tiles);
  // grouped order: kGroupM tile rows walked column by column
  const int group = t / (kGroupM * tiles_n);
  const int first_m = group * kGroupM;
  const int gm = min(tiles_m - first_m, kGroupM);
  const int in_group = t - group * kGroupM * tiles_n;
  const int tile_m = first_m + in_group % gm;
  const int tile_n = in_group / gm;
  const int m0 = tile_m * BM, n0 = tile_n * BN;

  gemm_tile<BM, BN, BK, TM, TN, T, VEC>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, m0, n0, As, Bs);
}

struct Config {
  int bm, bn;
};

// Tile configurations, in the order the autotuner and the parity tests see them.
constexpr Config kConfigs[] = {{128, 128}, {128, 256}, {256, 128}, {64, 64}};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

template <int BM, int BN, int BK, int TM, int TN, int MINB, typename T>
hipError_t launch_one(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B,
                      int64_t ldb, T *C, int64_t ldc, int accumulate, hipStream_t s) {
  const int tiles_m = (int)((M + BM - 1) / BM), tiles_n = (int)((N + BN - 1) / BN);
  const int num_tiles = tiles_m * tiles_n;
  constexpr int VE = 16 / sizeof(T);
  const bool vec = (lda % VE == 0) && (ldb % VE == 0) && (ldc % 2 == 0) &&
                   ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) &&
                   ((uintptr_t)C % 4 == 0);
  if (vec)
    hipLaunchKernelGGL((minplus_gemm_kernel<BM, BN, BK, TM, TN, MINB, T, true>), dim3(num_tiles),
                       dim3(kThreads), 0, s, (int)M, (int)N, (int)K, A, lda, B, ldb, C, ldc,
                       accumulate, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((minplus_gemm_kernel<BM, BN, BK, TM, TN, MINB, T, false>), dim3(num_tiles),
                       dim3(kThreads), 0, s, (int)M, (int)N, (int)K, A, lda, B, ldb, C, ldc,
                       accumulate, tiles_m, tiles_n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B,
                        int64_t ldb, T *C, int64_t ldc, int accumulate, int config,
                        hipStream_t s) {
  switch (config) {
    case 0:
      return launch_one<128, 128, 32, 8, 8, 4, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, s);
    case 1:
      return launch_one<128, 256, 32, 8, 16, 3, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, s);
    case 2:
      return launch_one<256, 128, 32, 16, 8, 3, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, s);
    default:
      return launch_one<64, 64, 32, 4, 4, 4, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, s);
  }
}

}  // namespace

int gemm_config_count() { return kNumConfigs; }

hipError_t launch_gemm(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                       const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                       int config, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (config < 0) {
    // default choice: large tiles when they fill the chip, small ones otherwise
    const int64_t big_tiles = ((M + 127) / 128) * ((N + 255) / 256);
    config = big_tiles >= 512 ? 1 : (((M + 127) / 128) * ((N + 127) / 128) >= 256 ? 0 : 3);
  }
  if (dtype == TP_U16)
    return launch_typed<uint16_t>(M, N, K, (const uint16_t *)A, lda, (const uint16_t *)B, ldb,
                                  (uint16_t *)C, ldc, accumulate, config, s);
  return launch_typed<uint8_t>(M, N, K, (const uint8_t *)A, lda, (const uint8_t *)B, ldb,
                               (uint8_t *)C, ldc, accumulate, config, s);
}

}  // namespace tp
