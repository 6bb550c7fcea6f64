// (min,+) matrix-vector products (Section 1 semiring; the companion work
// solves the small-cycle problem with these, and the walk along the path
// over cyclic columns runs on the vector-matrix form):
//   trans = 0:  y_i = min_k a_ik + x_k
//   trans = 1:  y_k = min_i x_i + a_ik
// Both read the matrix once and do two operations per 2-byte entry, so they
// are bound by HBM bandwidth.  With 16-bit entries, 16-byte aligned rows
// (lda a multiple of 8) and aligned vectors, every lane moves 16 bytes per
// load and works on packed pairs (v_pk_add_u16 with clamp, v_pk_min_u16);
// otherwise an element-wise kernel of the same results runs.
#include <algorithm>

#include "common.hpp"

namespace tp {

namespace {

template <typename T>
constexpr uint16_t inf_of() {
  return sizeof(T) == 2 ? 0xFFFFu : 0xFFu;
}

// ---------------------------------------------------------- element-wise --

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

// 16 waves split the rows, each lane owns two adjacent columns; the partial
// minima meet in LDS.  128 columns per workgroup.
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

// ------------------------------------------------------ 16-byte, 16-bit --

__device__ __forceinline__ void min_into(u16x2 (&acc)[4], uint4 a, uint4 b) {
  acc[0] = pk_min(acc[0], pk_add_sat(as_pk(a.x), as_pk(b.x)));
  acc[1] = pk_min(acc[1], pk_add_sat(as_pk(a.y), as_pk(b.y)));
  acc[2] = pk_min(acc[2], pk_add_sat(as_pk(a.z), as_pk(b.z)));
  acc[3] = pk_min(acc[3], pk_add_sat(as_pk(a.w), as_pk(b.w)));
}

// trans = 0: one wave per row; lane l reads entries 8l..8l+7 of every
// 512-entry stretch of the row and of x (x stays in cache: every row reads
// it), two stretches in flight per step; the row's tail below a whole
// 8-entry chunk is read element by element.
__global__ void __launch_bounds__(256) gemv_rows_vec_kernel(int64_t M, int64_t K,
                                                            const uint16_t *__restrict__ A,
                                                            int64_t lda,
                                                            const uint16_t *__restrict__ x,
                                                            uint16_t *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;
  gconst<uint16_t> row = to_global(A + i * lda);
  gconst<uint16_t> xv = to_global(x);
  const int64_t K8 = K & ~(int64_t)7;  // entries in whole 8-entry chunks
  u16x2 acc[4] = {splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu)};
  int64_t k = (int64_t)lane * 8;
  for (; k + 512 < K8; k += 1024) {
    const uint4 a0 = gload16<uint16_t>(row + k), a1 = gload16<uint16_t>(row + k + 512);
    const uint4 b0 = gload16<uint16_t>(xv + k), b1 = gload16<uint16_t>(xv + k + 512);
    min_into(acc, a0, b0);
    min_into(acc, a1, b1);
  }
  if (k < K8) min_into(acc, gload16<uint16_t>(row + k), gload16<uint16_t>(xv + k));
  u16x2 m2 = pk_min(pk_min(acc[0], acc[1]), pk_min(acc[2], acc[3]));
  uint32_t best = min((uint32_t)m2.x, (uint32_t)m2.y);
  for (int64_t t = K8 + lane; t < K; t += 64)
    best = min(best, min((uint32_t)row[t] + (uint32_t)xv[t], 0xFFFFu));
  for (int off = 32; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off));
  if (lane == 0) y[i] = (uint16_t)best;
}

// trans = 1: lane l of every wave owns columns 8l..8l+7 of the workgroup's
// 512-column stretch; the 16 waves split the workgroup's rows (four rows in
// flight per wave), x_r is one scalar load per row, and the 16 partial minima
// meet in LDS.  With one row group (gridDim.y == 1) the minima are stored;
// with several, each group folds its minima into y (filled with INF before)
// by a compare-and-swap of the packed pair per 32-bit word, so the whole chip
// works on a matrix with few 512-column stretches.  Columns past the last
// whole 8-entry chunk are read element by element.
__device__ __forceinline__ void fold_pair(uint16_t *y, u16x2 v) {
  unsigned int *w = reinterpret_cast<unsigned int *>(y);
  unsigned int old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (true) {
    const unsigned int want = as_u32(pk_min(as_pk(old), v));
    if (want == old) break;
    const unsigned int seen = atomicCAS(w, old, want);
    if (seen == old) break;
    old = seen;
  }
}

__global__ void __launch_bounds__(1024) gemv_cols_vec_kernel(int64_t M, int64_t K,
                                                             const uint16_t *__restrict__ A,
                                                             int64_t lda,
                                                             const uint16_t *__restrict__ x,
                                                             uint16_t *__restrict__ y,
                                                             int64_t rows_per_group) {
  __shared__ uint4 part[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = ((int64_t)blockIdx.x * 64 + lane) * 8;
  const int64_t r_begin = (int64_t)blockIdx.y * rows_per_group;
  const int64_t r_end = min(M, r_begin + rows_per_group);
  const bool whole = c + 8 <= K;
  gconst<uint16_t> a = to_global(A + c);
  u16x2 acc[4] = {splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu)};
  if (whole) {
    int64_t r = r_begin + wave;
    for (; r + 48 < r_end; r += 64) {
      const uint4 v0 = gload16<uint16_t>(a + r * lda), v1 = gload16<uint16_t>(a + (r + 16) * lda);
      const uint4 v2 = gload16<uint16_t>(a + (r + 32) * lda);
      const uint4 v3 = gload16<uint16_t>(a + (r + 48) * lda);
      const uint32_t x0 = x[r] * 0x10001u, x1 = x[r + 16] * 0x10001u;
      const uint32_t x2 = x[r + 32] * 0x10001u, x3 = x[r + 48] * 0x10001u;
      min_into(acc, v0, uint4{x0, x0, x0, x0});
      min_into(acc, v1, uint4{x1, x1, x1, x1});
      min_into(acc, v2, uint4{x2, x2, x2, x2});
      min_into(acc, v3, uint4{x3, x3, x3, x3});
    }
    for (; r < r_end; r += 16) {
      const uint32_t xx = x[r] * 0x10001u;
      min_into(acc, gload16<uint16_t>(a + r * lda), uint4{xx, xx, xx, xx});
    }
  } else if (c < K) {
    for (int64_t r = r_begin + wave; r < r_end; r += 16) {
      const uint32_t xr = x[r];
      for (int e = 0; e < 8 && c + e < K; ++e) {
        const uint16_t v = (uint16_t)min((uint32_t)A[r * lda + c + e] + xr, 0xFFFFu);
        u16x2 &slot = acc[e >> 1];
        slot = (e & 1) ? u16x2{slot.x, (uint16_t)min((uint32_t)slot.y, (uint32_t)v)}
                       : u16x2{(uint16_t)min((uint32_t)slot.x, (uint32_t)v), slot.y};
      }
    }
  }
  part[wave][lane] = uint4{as_u32(acc[0]), as_u32(acc[1]), as_u32(acc[2]), as_u32(acc[3])};
  __syncthreads();
  if (wave == 0 && c < K) {
    for (int w = 1; w < 16; ++w) {
      const uint4 p = part[w][lane];
      acc[0] = pk_min(acc[0], as_pk(p.x));
      acc[1] = pk_min(acc[1], as_pk(p.y));
      acc[2] = pk_min(acc[2], as_pk(p.z));
      acc[3] = pk_min(acc[3], as_pk(p.w));
    }
    if (gridDim.y == 1) {
      if (whole) {
        *reinterpret_cast<uint4 *>(y + c) =
            uint4{as_u32(acc[0]), as_u32(acc[1]), as_u32(acc[2]), as_u32(acc[3])};
      } else {
        for (int e = 0; c + e < K; ++e) y[c + e] = (e & 1) ? acc[e >> 1].y : acc[e >> 1].x;
      }
    } else {
      // whole pairs of columns only: with K odd the last column shares its
      // 32-bit word with the entry past the end of y, and is left to
      // gemv_last_col_kernel
      for (int t = 0; t < 4 && c + 2 * t + 1 < K; ++t) fold_pair(y + c + 2 * t, acc[t]);
    }
  }
}

// One column of the vector-matrix product by one workgroup: y_k = min_i x_i
// + a_ik (the last column of an odd K when row groups fold their minima).
__global__ void __launch_bounds__(1024) gemv_last_col_kernel(int64_t M,
                                                             const uint16_t *__restrict__ a,
                                                             int64_t lda,
                                                             const uint16_t *__restrict__ x,
                                                             uint16_t *__restrict__ y) {
  __shared__ uint32_t red[16];
  uint32_t best = 0xFFFFu;
  // sixteen rows in flight per lane: the column's entries are a cache line
  // apart each
  for (int64_t r0 = threadIdx.x; r0 < M; r0 += 1024 * 16) {
    uint32_t v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int64_t r = r0 + (int64_t)j * 1024;
      v[j] = r < M ? (uint32_t)a[r * lda] + (uint32_t)x[r] : 0xFFFFu;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) best = min(best, min(v[j], 0xFFFFu));
  }
  for (int off = 32; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) best = min(best, red[w]);
    *y = (uint16_t)best;
  }
}

__global__ void fill_u16_kernel(uint16_t *p, int64_t count, uint16_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

hipError_t launch_gemv(int dtype, int64_t M, int64_t K, const void *A, int64_t lda,
                       const void *x, void *y, int trans, hipStream_t s) {
  const bool vec = dtype == TP_U16 && lda % 8 == 0 && aligned16(A) && aligned16(x) &&
                   (trans == 0 || aligned16(y));
  if (!trans) {
    if (M == 0) return hipSuccess;
    dim3 grid((unsigned)((M + 3) / 4));
    if (vec)
      hipLaunchKernelGGL(gemv_rows_vec_kernel, grid, dim3(256), 0, s, M, K, (const uint16_t *)A,
                         lda, (const uint16_t *)x, (uint16_t *)y);
    else if (dtype == TP_U16)
      hipLaunchKernelGGL(gemv_rows_kernel<uint16_t>, grid, dim3(256), 0, s, M, K,
                         (const uint16_t *)A, lda, (const uint16_t *)x, (uint16_t *)y);
    else
      hipLaunchKernelGGL(gemv_rows_kernel<uint8_t>, grid, dim3(256), 0, s, M, K,
                         (const uint8_t *)A, lda, (const uint8_t *)x, (uint8_t *)y);
    return hipGetLastError();
  }
  if (K == 0) return hipSuccess;
  if (vec) {
    // row groups of at least 256 rows until about 4096 workgroups keep the
    // chip busy with a short tail
    const int64_t stretches = (K + 511) / 512;
    const int64_t want = std::max<int64_t>(1, 4096 / stretches);
    const int64_t groups = std::max<int64_t>(1, std::min(want, M / 256));
    const int64_t per = (M + groups - 1) / groups;
    const int64_t g = (M + per - 1) / per;
    if (g > 1)
      hipLaunchKernelGGL(fill_u16_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s,
                         (uint16_t *)y, K, (uint16_t)0xFFFFu);
    hipLaunchKernelGGL(gemv_cols_vec_kernel, dim3((unsigned)stretches, (unsigned)g), dim3(1024),
                       0, s, M, K, (const uint16_t *)A, lda, (const uint16_t *)x, (uint16_t *)y,
                       per);
    if (g > 1 && (K & 1))
      hipLaunchKernelGGL(gemv_last_col_kernel, dim3(1), dim3(1024), 0, s, M,
                         (const uint16_t *)A + (K - 1), lda, (const uint16_t *)x,
                         (uint16_t *)y + (K - 1));
    return hipGetLastError();
  }
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
