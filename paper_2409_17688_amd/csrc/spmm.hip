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
// 16-byte chunk of columns; successors are walked with 8 row loads in flight
// per lane.  The successor list and labels are wave-uniform.  Workgroups are
// numbered so each XCD takes a contiguous range of rows of one panel.
#include "device_core.hpp"

namespace tp {

namespace {

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) spmm_kernel(int64_t rows, const int64_t *__restrict__ rowptr,
                                                   const uint32_t *__restrict__ col,
                                                   const uint8_t *__restrict__ z,
                                                   const T *__restrict__ X, int64_t ldx,
                                                   T *__restrict__ Y, int64_t ldy, int64_t ncols) {
  constexpr int VE = 16 / sizeof(T);
  const int lane = threadIdx.x & 63;
  // 1-D grid over (panel, group of 4 rows); each XCD gets a contiguous range,
  // so rows with long common prefixes (and many common successors) share an L2
  const int64_t groups = (rows + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t q = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (q >= rows) return;
  const int64_t c0 = (panel * 64 + lane) * VE;
  if (c0 < ncols) spmm_row_chunk<T, VEC>(rowptr, col, z, X, ldx, Y, ldy, ncols, q, c0);
}

// The same product for the state matrix itself, from its packed successor
// list (successor and label in one word, scalar loads) with two rounds of
// gathers in flight (gather_row_colz); same launch shape as spmm_kernel.
template <int U>
__global__ void __launch_bounds__(256) state_gather_kernel(int64_t rows,
                                                           const int64_t *__restrict__ rowptr,
                                                           const uint32_t *__restrict__ colz,
                                                           const int32_t *__restrict__ order,
                                                           const uint16_t *__restrict__ X,
                                                           int64_t ldx, uint16_t *__restrict__ Y,
                                                           int64_t ldy, int64_t ncols) {
  const int lane = threadIdx.x & 63;
  const int64_t groups = (rows + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t slot = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (slot >= rows) return;
  // rows in the given order (longest successor lists first), else in index order
  const int64_t q = order ? (int64_t)((kconst_i32)order)[slot] : slot;
  const int64_t c0 = (panel * 64 + lane) * 8;
  gather_row_colz<U>((kconst_i64)rowptr, (kconst_u32)colz, X, ldx, Y, ldy, ncols, q, c0);
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
  const int32_t inf = (int32_t)storage_inf<T>();
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
  dim3 grid((unsigned)(((rows + 3) / 4) * panels));
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

hipError_t launch_state_gather(int64_t rows, const int64_t *rowptr, const uint32_t *colz,
                               const int32_t *order, const uint16_t *X, int64_t ldx, uint16_t *Y,
                               int64_t ldy, int64_t ncols, hipStream_t s) {
  if (rows == 0 || ncols == 0) return hipSuccess;
  const int64_t panels = (ncols + 511) / 512;
  dim3 grid((unsigned)(((rows + 3) / 4) * panels));
  hipLaunchKernelGGL(state_gather_kernel<8>, grid, dim3(256), 0, s, rows, rowptr, colz, order, X,
                     ldx, Y, ldy, ncols);
  return hipGetLastError();
}

bool state_gather_fits(const void *X, int64_t ldx, const void *Y, int64_t ldy, int64_t ncols) {
  // 16-byte rows and chunks, and rows long enough for the last 8-entry chunk
  return ldx % 8 == 0 && ldy % 8 == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)Y % 16 == 0 &&
         ldx >= (ncols + 7) / 8 * 8;
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
