// Left multiplication by the sparse state matrix: Y = A(D_n) x X.
//
// A(D_n) has an arc label that depends only on the successor (Section 2.2:
// the number of zeros of p), so row q of the product is
//   Y[q][j] = min over successors p of q of (z_p + X[p][j]),
// a gather of whole rows of X, one saturating add of a per-row constant and a
// min.  Power chains (Algorithm 2, A^k = A x A^(k-1)) only ever need this
// left multiplication, which costs nnz(A) * ncols operations instead of the
// N^3 of a dense product; the state matrix has under 4 % non-INF entries from
// n = 8 on and 0.77 % at n = 12.
//
// Launch shape: each wave owns one output row and a panel of 64 lanes x one
// 16-byte chunk of columns; successors are walked with 4 row loads in flight
// per lane.  The successor list and labels are wave-uniform.
#include "common.hpp"

namespace tp {

namespace {

template <typename T>
__device__ __forceinline__ uint16_t inf16();
template <>
__device__ __forceinline__ uint16_t inf16<uint16_t>() {
  return 0xFFFFu;
}
template <>
__device__ __forceinline__ uint16_t inf16<uint8_t>() {
  return 0xFFu;
}

// 16 bytes of row `row` starting at column col, as packed 16-bit pairs.
template <typename T, bool VEC>
__device__ __forceinline__ void load_row_chunk(const T *__restrict__ X, int64_t ldx, int64_t row,
                                               int64_t col, int64_t ncols,
                                               u16x2 (&out)[16 / sizeof(T) / 2]) {
  constexpr int VE = 16 / sizeof(T);
  const T *p = X + row * ldx + col;
  if (VEC && col + VE <= ncols) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    if constexpr (sizeof(T) == 2) {
      out[0] = as_pk(v.x);
      out[1] = as_pk(v.y);
      out[2] = as_pk(v.z);
      out[3] = as_pk(v.w);
    } else {
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // bytes b0 b1 b2 b3 -> (b0, b1), (b2, b3) widened to 16 bits
        out[2 * e] = as_pk(__builtin_amdgcn_perm(0u, w[e], 0x0c010c00u));
        out[2 * e + 1] = as_pk(__builtin_amdgcn_perm(0u, w[e], 0x0c030c02u));
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < VE / 2; ++e) {
      const int64_t c0 = col + 2 * e, c1 = c0 + 1;
      const uint16_t x0 = c0 < ncols ? (uint16_t)p[2 * e] : inf16<T>();
      const uint16_t x1 = c1 < ncols ? (uint16_t)p[2 * e + 1] : inf16<T>();
      out[e] = u16x2{x0, x1};
    }
  }
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) spmm_kernel(int64_t rows, const int64_t *__restrict__ rowptr,
                                                   const uint32_t *__restrict__ col,
                                                   const uint8_t *__restrict__ z,
                                                   const T *__restrict__ X, int64_t ldx,
                                                   T *__restrict__ Y, int64_t ldy, int64_t ncols) {
  constexpr int VE = 16 / sizeof(T);
  constexpr int P = VE / 2;  // packed registers per lane
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (q >= rows) return;
  const int64_t c0 = ((int64_t)blockIdx.y * 64 + lane) * VE;
  const int64_t begin = rowptr[q], end = rowptr[q + 1];
  u16x2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = splat(0xFFFFu);
  if (c0 < ncols) {
    int64_t e = begin;
    for (; e + 4 <= end; e += 4) {
      u16x2 v[4][P];
      uint16_t lab[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t p = col[e + u];
        lab[u] = z[p];
        load_row_chunk<T, VEC>(X, ldx, p, c0, ncols, v[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < P; ++r) acc[r] = pk_min(acc[r], pk_add_sat(splat(lab[u]), v[u][r]));
    }
    for (; e < end; ++e) {
      const uint32_t p = col[e];
      u16x2 v[P];
      load_row_chunk<T, VEC>(X, ldx, p, c0, ncols, v);
      const uint16_t lab = z[p];
#pragma unroll
      for (int r = 0; r < P; ++r) acc[r] = pk_min(acc[r], pk_add_sat(splat(lab), v[r]));
    }
    T *yrow = Y + q * ldy + c0;
    if constexpr (sizeof(T) == 1) {
#pragma unroll
      for (int r = 0; r < P; ++r) acc[r] = pk_min(acc[r], splat(0xFFu));
    }
    if (VEC && c0 + VE <= ncols) {
      uint4 w;
      if constexpr (sizeof(T) == 2) {
        w = uint4{as_u32(acc[0]), as_u32(acc[1]), as_u32(acc[2]), as_u32(acc[3])};
      } else {
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          o[k] = __builtin_amdgcn_perm(as_u32(acc[2 * k + 1]), as_u32(acc[2 * k]), 0x06040200u);
        w = uint4{o[0], o[1], o[2], o[3]};
      }
      *reinterpret_cast<uint4 *>(yrow) = w;
    } else {
#pragma unroll
      for (int r = 0; r < P; ++r) {
        if (c0 + 2 * r < ncols) yrow[2 * r] = (T)acc[r].x;
        if (c0 + 2 * r + 1 < ncols) yrow[2 * r + 1] = (T)acc[r].y;
      }
    }
  }
}

// min over arcs q -> p of z_p + X[p][q], one wave per row q, reduced into *out.
template <typename T>
__global__ void __launch_bounds__(256) sparse_trace_kernel(int64_t N,
                                                          const int64_t *__restrict__ rowptr,
                                                          const uint32_t *__restrict__ col,
                                                          const uint8_t *__restrict__ z,
                                                          const T *__restrict__ X, int64_t ldx,
                                                          int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int32_t inf = (int32_t)inf16<T>();
  int32_t best = inf;
  if (q < N) {
    for (int64_t e = rowptr[q] + lane; e < rowptr[q + 1]; e += 64) {
      const uint32_t p = col[e];
      const int32_t v = (int32_t)X[(int64_t)p * ldx + q] + (int32_t)z[p];
      best = min(best, min(v, inf));
    }
  }
  for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
  if (lane == 0 && best < inf) atomicMin(out, best);
}

template <typename T>
hipError_t launch_spmm_t(int64_t rows, const int64_t *rowptr, const uint32_t *col,
                         const uint8_t *z, const T *X, int64_t ldx, T *Y, int64_t ldy,
                         int64_t ncols, hipStream_t s) {
  constexpr int VE = 16 / sizeof(T);
  const int64_t panels = (ncols + 64 * VE - 1) / (64 * VE);
  dim3 grid((unsigned)((rows + 3) / 4), (unsigned)panels);
  const bool vec = (ldx % VE == 0) && (ldy % VE == 0) && ((uintptr_t)X % 16 == 0) &&
                   ((uintptr_t)Y % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((spmm_kernel<T, true>), grid, dim3(256), 0, s, rows, rowptr, col, z, X, ldx,
                       Y, ldy, ncols);
  else
    hipLaunchKernelGGL((spmm_kernel<T, false>), grid, dim3(256), 0, s, rows, rowptr, col, z, X,
                       ldx, Y, ldy, ncols);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_spmm(int dtype, int64_t rows, const int64_t *rowptr, const uint32_t *col,
                       const uint8_t *z, const void *X, int64_t ldx, void *Y, int64_t ldy,
                       int64_t ncols, hipStream_t s) {
  if (rows == 0 || ncols == 0) return hipSuccess;
  if (dtype == TP_U16)
    return launch_spmm_t<uint16_t>(rows, rowptr, col, z, (const uint16_t *)X, ldx, (uint16_t *)Y,
                                   ldy, ncols, s);
  return launch_spmm_t<uint8_t>(rows, rowptr, col, z, (const uint8_t *)X, ldx, (uint8_t *)Y, ldy,
                                ncols, s);
}

hipError_t launch_sparse_trace(int dtype, int64_t N, const int64_t *rowptr, const uint32_t *col,
                               const uint8_t *z, const void *X, int64_t ldx, int32_t *out,
                               hipStream_t s) {
  if (N == 0) return hipSuccess;
  dim3 grid((unsigned)((N + 3) / 4));
  if (dtype == TP_U16)
    hipLaunchKernelGGL(sparse_trace_kernel<uint16_t>, grid, dim3(256), 0, s, N, rowptr, col, z,
                       (const uint16_t *)X, ldx, out);
  else
    hipLaunchKernelGGL(sparse_trace_kernel<uint8_t>, grid, dim3(256), 0, s, N, rowptr, col, z,
                       (const uint8_t *)X, ldx, out);
  return hipGetLastError();
}

}  // namespace tp
