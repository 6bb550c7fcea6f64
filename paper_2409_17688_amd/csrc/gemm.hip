// Dense (min,+) matrix product C = A x B (Section 1: (A x B)_ij =
// min_k a_ik + b_kj), the product Algorithm 2 repeats for every power.
//
// The tile arithmetic lives in gemm_core.hpp.  This file launches one
// workgroup per tile, numbered so that each XCD (the hardware deals
// workgroups to the 8 XCDs in turn) gets a contiguous range of tiles, walked
// in groups of 8 tile rows, to keep A and B slabs shared in that XCD's L2.
//
// Split-K: when the output has too few tiles to fill the chip, K is cut into
// S slices (a second grid dimension); slice z writes the partial product
// over its K range to its own scratch matrix, and a reduction takes the
// elementwise min of the S partials (and of the old C when accumulating).
// This is exact: min over K = min over slices of min over the slice.
//
// The default choice of tile configuration and split comes from a table
// filled by the autotuner (keyed by the largest of M, N, K), else from a
// heuristic.
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

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
                        int accumulate, int tiles_m, int tiles_n, int kslice,
                        int64_t slice_stride) {
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
  // K slice of this workgroup (the whole K without a split)
  const int k0 = (int)blockIdx.y * kslice;
  const int kl = min(K - k0, kslice);
  gemm_tile<BM, BN, BK, TM, TN, T, VEC>(M, N, kl, A + k0, lda, B + (int64_t)k0 * ldb, ldb,
                                        C + (int64_t)blockIdx.y * slice_stride, ldc, accumulate,
                                        m0, n0, As, Bs);
}

// C = min over the S partial products (and the old C when accumulating).
template <typename T>
__global__ void __launch_bounds__(256) ksplit_reduce_kernel(int64_t M, int64_t N,
                                                            const T *__restrict__ W, int64_t ldw,
                                                            int64_t slice_stride, int S,
                                                            T *__restrict__ C, int64_t ldc,
                                                            int accumulate) {
  const int64_t total = M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / N, c = i - r * N;
    T v = W[r * ldw + c];
    for (int z = 1; z < S; ++z) v = min(v, W[z * slice_stride + r * ldw + c]);
    if (accumulate) v = min(v, C[r * ldc + c]);
    C[r * ldc + c] = v;
  }
}

struct Config {
  int bm, bn;
};

// Tile configurations, in the order the autotuner and the parity tests see them.
constexpr Config kConfigs[] = {{128, 128}, {128, 256}, {256, 128}, {64, 64}, {256, 256}};
constexpr int kNumConfigs = sizeof(kConfigs) / sizeof(kConfigs[0]);

// Launches the product with S K-slices of kslice columns each (S = 1: no
// split, C written directly; S > 1: partials into W, slice z at
// W + z * slice_stride with leading dimension ldw).
template <int BM, int BN, int BK, int TM, int TN, int MINB, typename T>
hipError_t launch_one(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B,
                      int64_t ldb, T *C, int64_t ldc, int accumulate, int S, int64_t kslice,
                      T *W, int64_t ldw, int64_t slice_stride, hipStream_t s) {
  const int tiles_m = (int)((M + BM - 1) / BM), tiles_n = (int)((N + BN - 1) / BN);
  const int num_tiles = tiles_m * tiles_n;
  constexpr int VE = 16 / sizeof(T);
  T *out = S > 1 ? W : C;
  const int64_t ldo = S > 1 ? ldw : ldc;
  const bool vec = (lda % VE == 0) && (ldb % VE == 0) && (ldo % 2 == 0) &&
                   ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) &&
                   ((uintptr_t)out % 4 == 0);
  const dim3 grid(num_tiles, S);
  const int ks = S > 1 ? (int)kslice : (int)K;
  const int acc = S > 1 ? 0 : accumulate;
  const int64_t stride = S > 1 ? slice_stride : 0;
  if (vec)
    hipLaunchKernelGGL((minplus_gemm_kernel<BM, BN, BK, TM, TN, MINB, T, true>), grid,
                       dim3(kThreads), 0, s, (int)M, (int)N, (int)K, A, lda, B, ldb, out, ldo,
                       acc, tiles_m, tiles_n, ks, stride);
  else
    hipLaunchKernelGGL((minplus_gemm_kernel<BM, BN, BK, TM, TN, MINB, T, false>), grid,
                       dim3(kThreads), 0, s, (int)M, (int)N, (int)K, A, lda, B, ldb, out, ldo,
                       acc, tiles_m, tiles_n, ks, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  const int64_t total = M * N;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(ksplit_reduce_kernel<T>, dim3(blocks), dim3(256), 0, s, M, N,
                     (const T *)W, ldw, slice_stride, S, C, ldc, accumulate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B,
                        int64_t ldb, T *C, int64_t ldc, int accumulate, int config, int S,
                        int64_t kslice, T *W, int64_t ldw, int64_t stride, hipStream_t s) {
  switch (config) {
    case 0:
      return launch_one<128, 128, 32, 8, 8, 4, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, S,
                                                  kslice, W, ldw, stride, s);
    case 1:
      return launch_one<128, 256, 32, 8, 16, 3, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, S,
                                                   kslice, W, ldw, stride, s);
    case 2:
      return launch_one<256, 128, 32, 16, 8, 3, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, S,
                                                   kslice, W, ldw, stride, s);
    case 4:
      return launch_one<256, 256, 32, 16, 16, 2, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate,
                                                    S, kslice, W, ldw, stride, s);
    default:
      return launch_one<64, 64, 32, 4, 4, 4, T>(M, N, K, A, lda, B, ldb, C, ldc, accumulate, S,
                                                kslice, W, ldw, stride, s);
  }
}

// Scratch for split-K partials, one grow-only buffer per (device, stream):
// calls on one stream run in order, so they can share it.
struct Scratch {
  void *p = nullptr;
  size_t bytes = 0;
};
std::mutex g_scratch_mu;
std::map<std::pair<int, hipStream_t>, Scratch> g_scratch;

hipError_t scratch_for(hipStream_t s, size_t bytes, void **out) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  Scratch &sc = g_scratch[{dev, s}];
  if (sc.bytes < bytes) {
    if (sc.p) {
      // the old buffer may still be read by queued work on this stream
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      e = hipFree(sc.p);
      if (e != hipSuccess) return e;
      sc.p = nullptr;
      sc.bytes = 0;
    }
    hipError_t e = hipMalloc(&sc.p, bytes);
    if (e != hipSuccess) return e;
    sc.bytes = bytes;
  }
  *out = sc.p;
  return hipSuccess;
}

// Autotuned defaults per dtype: entries (max_dim, config, ksplit) sorted by
// max_dim; a product uses the first entry with max(M, N, K) <= max_dim.
struct Choice {
  int64_t max_dim;
  int config, ksplit;
};
std::mutex g_tune_mu;
std::vector<Choice> g_tune[2];

int dtype_index(int dtype) { return dtype == TP_U16 ? 0 : 1; }

}  // namespace

int gemm_tune_set(int dtype, int64_t max_dim, int config, int ksplit) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::vector<Choice> &t = g_tune[dtype_index(dtype)];
  if (max_dim < 0) {
    t.clear();
    return TP_OK;
  }
  for (Choice &c : t)
    if (c.max_dim == max_dim) {
      c.config = config;
      c.ksplit = ksplit;
      return TP_OK;
    }
  t.push_back({max_dim, config, ksplit});
  std::sort(t.begin(), t.end(), [](const Choice &a, const Choice &b) { return a.max_dim < b.max_dim; });
  return TP_OK;
}

void gemm_choice(int dtype, int64_t M, int64_t N, int64_t K, int *config, int *ksplit) {
  const int64_t key = std::max(M, std::max(N, K));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const Choice &c : g_tune[dtype_index(dtype)])
      if (key <= c.max_dim) {
        *config = c.config;
        *ksplit = c.ksplit;
        return;
      }
  }
  // heuristic: large tiles when they fill the chip, small ones otherwise;
  // split K when even small tiles leave most of the chip idle
  const int64_t big_tiles = ((M + 127) / 128) * ((N + 255) / 256);
  const int64_t tiles128 = ((M + 127) / 128) * ((N + 127) / 128);
  const int64_t tiles64 = ((M + 63) / 64) * ((N + 63) / 64);
  *config = big_tiles >= 512 ? 1 : (tiles128 >= 256 ? 0 : 3);
  *ksplit = 1;
  if (*config == 3 && tiles64 < 256 && K >= 1024)
    *ksplit = (int)std::min<int64_t>(8, std::max<int64_t>(1, 512 / std::max<int64_t>(tiles64, 1)));
}

int gemm_config_count() { return kNumConfigs; }

namespace {

// Slices of a multiple of 64 columns (keeps the slices' 16-byte alignment).
void split_of(int64_t K, int ksplit, int *S, int64_t *kslice) {
  *S = 1;
  *kslice = K;
  if (ksplit > 1 && K > 64) {
    *kslice = ((K + ksplit - 1) / ksplit + 63) / 64 * 64;
    *S = (int)((K + *kslice - 1) / *kslice);
  }
}

int64_t partial_ld(int64_t N) { return (N + 63) / 64 * 64; }

size_t partial_bytes(int dtype, int64_t M, int64_t N, int S) {
  return (size_t)S * (size_t)M * (size_t)partial_ld(N) * (dtype == TP_U16 ? 2 : 1);
}

// The product with S slices of kslice columns, partials (S > 1) in W.
hipError_t launch_split(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                        const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                        int config, int S, int64_t kslice, void *W, hipStream_t s) {
  const int64_t ldw = S > 1 ? partial_ld(N) : 0, stride = S > 1 ? M * ldw : 0;
  if (dtype == TP_U16)
    return launch_typed<uint16_t>(M, N, K, (const uint16_t *)A, lda, (const uint16_t *)B, ldb,
                                  (uint16_t *)C, ldc, accumulate, config, S, kslice,
                                  (uint16_t *)W, ldw, stride, s);
  return launch_typed<uint8_t>(M, N, K, (const uint8_t *)A, lda, (const uint8_t *)B, ldb,
                               (uint8_t *)C, ldc, accumulate, config, S, kslice, (uint8_t *)W,
                               ldw, stride, s);
}

}  // namespace

hipError_t launch_gemm(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                       const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                       int config, int ksplit, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (config < 0) {
    // tuned shape; ksplit 0 keeps it unsplit (no scratch: nothing allocated)
    int tuned_split = 1;
    gemm_choice(dtype, M, N, K, &config, &tuned_split);
    ksplit = ksplit == 0 ? 1 : tuned_split;
  }
  int S = 1;
  int64_t kslice = K;
  split_of(K, ksplit, &S, &kslice);
  void *W = nullptr;
  if (S > 1) {
    hipError_t e = scratch_for(s, partial_bytes(dtype, M, N, S), &W);
    if (e != hipSuccess) return e;
  }
  return launch_split(dtype, M, N, K, A, lda, B, ldb, C, ldc, accumulate, config, S, kslice, W,
                      s);
}

// --------------------------------------------------------------------------
// Fixed scratch for callers that cannot allocate (code under graph capture,
// tight serving loops): the split-K partials go to this file-scope array,
// one copy per device, held until the process ends.  Its name on the host is
// a stand-in for the symbol, not a device address: host code reaches the
// memory only through the address hipGetSymbolAddress gives for the current
// device, kept per device below.
static __device__ __align__(256) uint8_t scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {nullptr};

hipError_t fixed_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_fixed_ptr[dev] = p;
  }
  *out = g_fixed_ptr[dev];
  return hipSuccess;
}
}  // namespace

int launch_gemm_fixed(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                      const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                      int config, int ksplit, hipStream_t s) {
  int S = 1;
  int64_t kslice = K;
  split_of(K, ksplit, &S, &kslice);
  void *W = nullptr;
  if (S > 1 && M > 0 && N > 0) {
    const size_t need = partial_bytes(dtype, M, N, S);
    if (need > kFixedScratchBytes) {
      set_error("%d K slices of a %lld x %lld product need %zu bytes of scratch; the fixed "
                "buffer holds %zu",
                S, (long long)M, (long long)N, need, kFixedScratchBytes);
      return TP_EINVAL;
    }
    TP_HIP_CHECK(fixed_scratch(&W));
  }
  if (M == 0 || N == 0) return TP_OK;
  TP_HIP_CHECK(launch_split(dtype, M, N, K, A, lda, B, ldb, C, ldc, accumulate, config, S, kslice,
                            W, s));
  return TP_OK;
}

}  // namespace tp
