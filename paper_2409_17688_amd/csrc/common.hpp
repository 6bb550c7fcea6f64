// Internal helpers shared by the HIP translation units of libtropical.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "tropical.h"

namespace tp {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

constexpr uint16_t kInf16 = 0xFFFFu;
constexpr uint8_t kInf8 = 0xFFu;

// Saturating packed add and packed min: one v_pk_add_u16 (clamp) and one
// v_pk_min_u16 per two lanes of 16-bit entries.  With entries in [0, INF]
// the clamp makes INF absorbing, which is the semiring's rule a + INF = INF.
__device__ __forceinline__ u16x2 pk_add_sat(u16x2 a, u16x2 b) {
  return __builtin_elementwise_add_sat(a, b);
}
__device__ __forceinline__ u16x2 pk_min(u16x2 a, u16x2 b) {
  return __builtin_elementwise_min(a, b);
}
__device__ __forceinline__ u16x2 splat(uint16_t v) { return u16x2{v, v}; }

// The hardware deals consecutive workgroups to the 8 XCDs in turn.  This maps
// the workgroup id to a work index such that each XCD receives a contiguous
// range of [0, total) (a bijection), so neighbouring work shares an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t total) {
  const int64_t q = total >> 3, r = total & 7;
  const int64_t x = bid & 7, local = bid >> 3;
  return x * q + (x < r ? x : r) + local;
}

__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 as_pk(uint32_t v) { return __builtin_bit_cast(u16x2, v); }

// Every matrix this library touches lives in global memory.  A pointer that
// reaches a kernel through memory (a task table) is a generic one to the
// compiler, whose loads become flat loads with per-lane 64-bit addresses and
// waits shared with LDS traffic; reading through these views keeps them
// global loads wherever the pointer came from.  (Index in the global space:
// offsetting the generic pointer first lets the cast be folded away.)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
using gconst = const __attribute__((address_space(1))) T *;
template <typename T>
using gmut = __attribute__((address_space(1))) T *;

// Read-only tables (the resident CSR): through constant-space views a
// wave-uniform index becomes a scalar load.
typedef const __attribute__((address_space(4))) int64_t *kconst_i64;
typedef const __attribute__((address_space(4))) int32_t *kconst_i32;
typedef const __attribute__((address_space(4))) uint32_t *kconst_u32;
typedef const __attribute__((address_space(4))) uint64_t *kconst_u64;

// A value the whole wave holds the same copy of, moved to scalar registers.
// A pointer loaded from memory (a slot table) lives in vector registers to
// the compiler even when every lane loaded the same one, and loads through
// it then stay per-lane vector loads that wait for each other; made scalar,
// loads through constant-space views of it become scalar loads again.
template <typename T>
__device__ __forceinline__ T *wave_uniform(T *p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T *)(uintptr_t)(hi << 32 | lo);
}
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const uint64_t v = (uint64_t)x;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (int64_t)(hi << 32 | lo);
}

template <typename T>
__device__ __forceinline__ gconst<T> to_global(const T *p) {
  return (gconst<T>)p;
}
template <typename T>
__device__ __forceinline__ gmut<T> to_global_mut(T *p) {
  return (gmut<T>)p;
}
// 16 and 8 bytes at global element address p (aligned).
template <typename T>
__device__ __forceinline__ uint4 gload16(gconst<T> p) {
  const u32x4 v = *(gconst<u32x4>)p;
  return uint4{v.x, v.y, v.z, v.w};
}
template <typename T>
__device__ __forceinline__ uint2 gload8(gconst<T> p) {
  const u32x2 v = *(gconst<u32x2>)p;
  return uint2{v.x, v.y};
}

// Host side: status plumbing.
void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

}  // namespace tp

#define TP_HIP_CHECK(expr)                                   \
  do {                                                       \
    hipError_t tp_e_ = (expr);                               \
    if (tp_e_ != hipSuccess) return tp::hip_fail(tp_e_, #expr); \
  } while (0)

#define TP_REQUIRE(cond, ...)           \
  do {                                  \
    if (!(cond)) {                      \
      tp::set_error(__VA_ARGS__);       \
      return TP_EINVAL;                 \
    }                                   \
  } while (0)

// Launchers implemented in the kernel translation units (host functions).
namespace tp {

// The row blocks of A(D_n) cut by rows into parts of bounded length, for
// the steps that give each part to one workgroup (the batch kernel's chain
// levels, the small-n step): part f has entries fptr[f] .. fptr[f+1]-1 of
// fent (the blocked layout, masks cut to the part's rows and grouped again),
// finfo[f] = block << 16 | the part's row mask; fptrh is fptr on the host.
// Built with the state for n <= 10, on first use above, and kept.
struct FineView {
  int64_t nf;
  const int64_t *fptr;
  const uint64_t *fent;
  const uint32_t *finfo;
  const int32_t *forder;  // parts by decreasing entry count (device)
  const int64_t *fptrh;
};
// Device-resident description of A(D_n) from the process-wide cache (api.hip);
// pointers stay valid until tp_release_cache.
struct StateView {
  int n;
  int64_t N, nnz;
  const uint32_t *masks;
  const int64_t *rowptr;
  const uint32_t *col;
  const uint8_t *z;
  const uint32_t *colz;  // col with z of each successor in the top byte
  // blocked form (16 rows per block): entries bptr[b] .. bptr[b+1]-1 of ent
  const int64_t *bptr;
  const uint64_t *bent;
  int64_t nent;
  const int32_t *order;   // rows by decreasing out-degree
  const int32_t *border;  // row blocks by decreasing entry count
  const int32_t *degh;    // host: out-degree of each row
  FineView fine;          // row-block parts (nf = 0 when not built)
};
int state_view(int n, hipStream_t s, StateView *out);
int state_fine_view(int n, hipStream_t s, FineView *out);
// The plain path's cost model for path order n (its tuned rates): seconds of
// one sparse left step (nnz N operations) and of one dense product (N^3).
void step_and_product_seconds(int n, double N, double nnz, double *step, double *product);
// Y = A(D_n) x X (u16) in the form the library picks for n (tp_tune_step).
hipError_t state_step_view(const StateView &v, const uint16_t *X, int64_t ldx, uint16_t *Y,
                           int64_t ldy, int64_t ncols, hipStream_t s);

// compact.hip: shared-base compact powers (u8 residuals, base[0] = G,
// base[1] = least residual; status bits 1 = range, 2 = INF present)
// Path orders from which the power chains of tp_recurrence and of the
// pruned plain path run on shared-base compact powers (0: never).
bool compact_chain(int n);
hipError_t launch_shared_to_u16(int64_t N, int64_t ncols, const uint8_t *X, int64_t ldx,
                                const int32_t *base, uint16_t *Y, int64_t ldy, hipStream_t s);
hipError_t launch_shared_from_u16(int64_t N, int64_t ncols, const uint16_t *X, int64_t ldx,
                                  uint8_t *Y, int64_t ldy, int32_t *base, int32_t *status,
                                  hipStream_t s);
hipError_t launch_shared_step(const StateView &v, const uint8_t *X, int64_t ldx, const int32_t *bx,
                              uint8_t *Y, int64_t ldy, int32_t *by, int64_t ncols,
                              int32_t *status, hipStream_t s);
hipError_t launch_shared_diag(int64_t N, const uint8_t *X, int64_t ldx, const int32_t *base,
                              int32_t *out, hipStream_t s);

// state.hip
int64_t word_count_host(int n);
hipError_t launch_words(int n, uint32_t *codes, uint8_t *zeros, uint32_t *masks, hipStream_t s);
hipError_t launch_dense_state(int n, int64_t N, const uint32_t *masks, int dtype, void *A,
                              int64_t lda, hipStream_t s);
hipError_t launch_csr_count(int64_t N, int n, const uint32_t *masks, int64_t *rowptr,
                            hipStream_t s);
hipError_t launch_scan_rowptr(int64_t N, int64_t *rowptr, hipStream_t s);
hipError_t launch_csr_fill(int64_t N, int n, const uint32_t *masks, const int64_t *rowptr,
                           uint32_t *col, uint32_t *colz, hipStream_t s);

// spmm.hip: the state matrix's own step from its packed successor list; rows
// in `order` (a permutation of 0..rows-1) when it is not NULL
hipError_t launch_state_gather(int64_t rows, const int64_t *rowptr, const uint32_t *colz,
                               const int32_t *order, const uint16_t *X, int64_t ldx, uint16_t *Y,
                               int64_t ldy, int64_t ncols, hipStream_t s);
bool state_gather_fits(const void *X, int64_t ldx, const void *Y, int64_t ldy, int64_t ncols);

// blockstep.hip: the sparse left step over blocks of 16 rows.  An entry of a
// block is p (bits 0..23), z_p (24..31), the mask of the block's rows that
// have p as a successor (32..47) and, in bit 48, the end of a run of entries
// with one mask (entries of a block are grouped by mask, then ordered by p)
constexpr uint64_t kGroupEnd = 1ull << 48;
int64_t block_count_host(int64_t N);
hipError_t launch_block_count(int64_t N, int n, const uint32_t *masks, int64_t *bptr,
                              hipStream_t s);
hipError_t launch_block_fill(int64_t N, int n, const uint32_t *masks, const int64_t *bptr,
                             uint64_t *ent, hipStream_t s);
// blocks in `border` (a permutation of the blocks) when it is not NULL
// (grouped: the entries a mask group at a time)
// `fine` (may be null): the row-block parts, which the grouped step takes
// where the blocks alone would leave the chip short of work (small n).
hipError_t launch_block_step(int64_t N, const int64_t *bptr, const uint64_t *ent,
                             const int32_t *border, const FineView *fine, const uint16_t *X,
                             int64_t ldx, uint16_t *Y, int64_t ldy, int64_t ncols, bool grouped,
                             hipStream_t s);

// gemm.hip
// config >= 0: that tile configuration with ksplit slices (>= 1); config < 0:
// the tuned shape, with its K split when ksplit < 0 and unsplit (so without
// scratch) when ksplit == 0
hipError_t launch_gemm(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                       const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                       int config, int ksplit, hipStream_t s);
// the same into the fixed per-device scratch (allocates nothing); a status:
// TP_EINVAL when the partials need more than kFixedScratchBytes
constexpr size_t kFixedScratchBytes = TP_NOALLOC_SCRATCH_BYTES;
int launch_gemm_fixed(int dtype, int64_t M, int64_t N, int64_t K, const void *A, int64_t lda,
                      const void *B, int64_t ldb, void *C, int64_t ldc, int accumulate,
                      int config, int ksplit, hipStream_t s);
// tuning table of the default (config < 0) choice; max_dim < 0 clears it
int gemm_tune_set(int dtype, int64_t max_dim, int config, int ksplit);
void gemm_choice(int dtype, int64_t M, int64_t N, int64_t K, int *config, int *ksplit);
int gemm_config_count();

// cyclic.hip: columns that are copies of the cycle C_m (3 <= m <= 12)
int64_t cyclic_count_host(int m);
hipError_t launch_cyclic_words(int m, uint32_t *codes, uint8_t *zeros, uint32_t *masks,
                               hipStream_t s);
hipError_t launch_cyclic_dense(int m, int64_t N, const uint32_t *masks, int dtype, void *A,
                               int64_t lda, hipStream_t s);
hipError_t launch_cyclic_boundary(int m, int64_t N, const uint32_t *masks, int dtype, void *start,
                                  void *end, hipStream_t s);
hipError_t launch_cyclic_pred_count(int m, int64_t N, const uint32_t *masks, int64_t *predptr,
                                    hipStream_t s);
hipError_t launch_cyclic_pred_fill(int m, int64_t N, const uint32_t *masks, const int64_t *predptr,
                                   uint16_t *pred, hipStream_t s);
int64_t cyclic_strip_length(int64_t nnz);
hipError_t launch_cyclic_strips(int64_t N, int64_t nnz, const int64_t *predptr,
                                const uint16_t *pred, uint32_t *strips, hipStream_t s);
hipError_t launch_cyclic_chain(int64_t N, int64_t nnz, int64_t nmax, const uint32_t *strips,
                               const uint8_t *z, const uint16_t *start, const uint16_t *end,
                               int32_t *out, hipStream_t s);
// the step form's work items (predecessor lists cut into pieces, longest
// lists first), as bytes to upload; returns their count
int64_t cyclic_items_host(int64_t N, const int64_t *predptr, const int32_t *order,
                          std::vector<char> *bytes);
hipError_t launch_cyclic_step(int64_t N, int64_t nitems, const void *items, const uint16_t *pred,
                              const uint8_t *z, const uint16_t *end, uint32_t *ym,
                              const uint16_t *x, uint16_t *y, int32_t *out, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s);
hipError_t launch_cyclic_answer(int64_t N, const uint16_t *x, const uint16_t *end, int32_t *out,
                                hipStream_t s);
// cyclic_api.hip: frees the cache of cyclic column digraphs
void cyclic_release_cache();

// gemv.hip
hipError_t launch_gemv(int dtype, int64_t M, int64_t K, const void *A, int64_t lda,
                       const void *x, void *y, int trans, hipStream_t s);

// spmm.hip
hipError_t launch_spmm(int dtype, int64_t rows, const int64_t *rowptr, const uint32_t *col,
                       const uint8_t *z, const void *X, int64_t ldx, void *Y, int64_t ldy,
                       int64_t ncols, hipStream_t s);
hipError_t launch_sparse_trace(int dtype, int64_t N, const int64_t *rowptr, const uint32_t *col,
                               const uint8_t *z, const void *X, int64_t ldx, int32_t *out,
                               hipStream_t s);

// trace.hip
hipError_t launch_fill_i32(int32_t *p, int64_t count, int32_t value, hipStream_t s);
hipError_t launch_fill_bytes(void *p, size_t count, uint8_t value, hipStream_t s);
// prune.hip: columns idx of A(D_n) as a dense u16 panel; min_j X[idx[j]][j]
hipError_t launch_state_columns(int n, int64_t N, const uint32_t *masks, const int32_t *idx,
                                int64_t count, uint16_t *X, int64_t ldx, hipStream_t s);
hipError_t launch_diag_select_min(int64_t rows, int64_t count, const int32_t *idx,
                                  const uint16_t *X, int64_t ldx, int32_t *out, hipStream_t s);
hipError_t launch_trace_min(int dtype, int64_t N, const void *X, int64_t ldx, int32_t *out,
                            hipStream_t s);
hipError_t launch_trace_of_product(int dtype, int64_t N, const void *X, int64_t ldx,
                                   const void *Y, int64_t ldy, int32_t *out, hipStream_t s);

}  // namespace tp
