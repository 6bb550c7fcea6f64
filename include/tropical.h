/*
 * tropical.h -- C ABI of libtropical.so: exact integer (min,+) matrix
 * arithmetic on an MI355X (gfx950) and the 2-domination number of cylinders
 * P_n x C_m by tropical matrix powers (arXiv 2409.17688).
 *
 * Notation: n is the order of the path (the paper's m), m the order of the
 * cycle (the paper's n).  The state matrix A(D_n) of Section 2.2 has one row
 * and one column per correct word of length n over {0,1,2}; words are indexed
 * in increasing order of their base-3 value with the first letter most
 * significant.  A[q][p] = number of zeros of p when p can follow q, else INF.
 *
 * Element types.  Matrices hold small non-negative integers in unsigned 8-bit
 * (INF = 255) or 16-bit (INF = 65535) storage.  Every value >= INF means INF;
 * sums saturate: a + b >= INF gives INF.  Results are exact: the semiring of
 * Section 1 on integers, with no rounding anywhere.
 *
 * Conventions for every call below.
 *   Layout     row-major; leading dimensions are in elements and >= the row
 *              length.  Pointers named d_* or documented as device pointers
 *              are device memory owned by the caller; the library never frees
 *              them.
 *   Streams    work is queued on `stream` (NULL = the default stream) and the
 *              call returns without waiting, unless stated otherwise.
 *   Errors     a negative TP_E* status; nothing is written or queued when the
 *              arguments are rejected (TP_EINVAL, TP_EOVERFLOW).  A failing
 *              HIP call gives TP_EHIP.  tp_last_error() returns a text for the
 *              last failure of the calling thread.
 *   Sizes      0 <= M, N, K < 2^31 elements per dimension; empty shapes are
 *              accepted and do nothing (an empty inner dimension gives INF).
 *   Aliasing   outputs must not overlap inputs unless stated otherwise.
 *   Determinism results are bit-identical for any tiling, launch shape or
 *              batching: min and saturating + on integers are exact.
 */
#ifndef TROPICAL_H
#define TROPICAL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* element types */
#define TP_U8 1  /* uint8_t, INF = 255 */
#define TP_U16 2 /* uint16_t, INF = 65535 */

/* status codes */
#define TP_OK 0
#define TP_EINVAL (-1)    /* bad argument: size, pointer, dtype, n or m      */
#define TP_ENOMEM (-2)    /* device memory or the context budget exhausted   */
#define TP_EOVERFLOW (-3) /* finite results could reach INF: n*m >= INF      */
#define TP_EHIP (-4)      /* a HIP runtime call failed                       */
#define TP_EBUSY (-5)     /* the context cannot take more work right now     */
#define TP_ECANCELED (-6) /* the request was cancelled before it ran         */

/* Text describing the calling thread's last failure ("" if none). */
const char *tp_last_error(void);

/* ABI version, currently 1. */
int tp_version(void);

/* ------------------------------------------------------------------------ */
/* State matrix A(D_n): Section 2.2 (correct words, the "can follow" rule,    */
/* arc label = zeros of the successor) and Algorithm 1 of Section 3.          */
/* ------------------------------------------------------------------------ */

/* N = |C_n|, the number of correct words of length n (Table 1), for
 * 1 <= n <= 13; TP_EINVAL otherwise.  Host-side count, no GPU work. */
int64_t tp_state_dim(int n);

/* Number of arcs of D_n (non-INF entries of A(D_n)), 1 <= n <= 13.  The first
 * call for a given n counts them on the current device and blocks; later
 * calls return a cached value.  Negative status on failure. */
int64_t tp_state_nnz(int n);

/* d_codes[0..N-1] = base-3 codes of the correct words of length n in
 * increasing order (device uint32_t array of N entries). */
int tp_words(int n, uint32_t *d_codes, hipStream_t stream);

/* Dense A(D_n) into d_A (N x N, leading dimension lda >= N), dtype TP_U8 or
 * TP_U16. */
int tp_build_state_matrix(int n, int dtype, void *d_A, int64_t lda, hipStream_t stream);

/* A(D_n) in compressed sparse rows.  d_rowptr: N+1 int64 (row q's arcs are
 * d_col[d_rowptr[q] .. d_rowptr[q+1]-1]), d_col: tp_state_nnz(n) uint32
 * successor indices in increasing order, d_z: N uint8 zero counts, so that
 * A[q][p] = d_z[p] for every stored p.  Any of d_col / d_z may be NULL to
 * skip it. */
int tp_build_state_csr(int n, int64_t *d_rowptr, uint32_t *d_col, uint8_t *d_z,
                       hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* (min,+) products: (A x B)_ij = min_k (a_ik + b_kj), Section 1.            */
/* ------------------------------------------------------------------------ */

/* C (M x N) = A (M x K) x B (K x N); with accumulate != 0,
 * C = min(C, A x B) elementwise.  Device pointers of the given dtype.  Runs
 * the tile configuration the tuning table gives for max(M, N, K), never with
 * a K split: it allocates nothing (the library's own products, and
 * tp_minplus_gemm_ex, may split K into scratch). */
int tp_minplus_gemm(int dtype, int64_t M, int64_t N, int64_t K,
                    const void *d_A, int64_t lda, const void *d_B, int64_t ldb,
                    void *d_C, int64_t ldc, int accumulate, hipStream_t stream);

/* Number of tile configurations of the dense product (for tuning). */
int tp_gemm_config_count(void);

/* tp_minplus_gemm with an explicit tile configuration 0 <= config <
 * tp_gemm_config_count(); every configuration gives the same result.  For an
 * autotuner and for tests that cover every configuration. */
int tp_minplus_gemm_config(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A,
                           int64_t lda, const void *d_B, int64_t ldb, void *d_C, int64_t ldc,
                           int accumulate, int config, hipStream_t stream);

/* tp_minplus_gemm_config with K split into up to ksplit slices (1 <= ksplit
 * <= 64; 1 = no split).  The slices (a multiple of 64 columns each) run as
 * separate workgroups whose partial products go to library-owned scratch
 * (one grow-only buffer per device and stream, allocated on first use, so
 * not for code under graph capture); a reduction kernel then writes C as
 * their elementwise minimum, and with accumulate != 0 the minimum with the
 * old C.  The result equals the unsplit product: min over K is the minimum
 * over the slices of the minimum within each.  Fills the chip when M x N
 * has few output tiles.  TP_EINVAL on a bad config or ksplit. */
int tp_minplus_gemm_ex(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A, int64_t lda,
                       const void *d_B, int64_t ldb, void *d_C, int64_t ldc, int accumulate,
                       int config, int ksplit, hipStream_t stream);

/* Bytes of the fixed split-K scratch of tp_minplus_gemm_ex_noalloc. */
#define TP_NOALLOC_SCRATCH_BYTES (64ll << 20)

/* tp_minplus_gemm_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same product, kernels and result, with the split-K
 * partials in a fixed buffer of TP_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends, instead of
 * scratch it allocates.  Allocates nothing and frees nothing.  The partials
 * of S slices take S * M * (N rounded up to 64) elements; a product whose
 * partials exceed the buffer is rejected with TP_EINVAL (nothing queued).
 * Every call on one device shares that buffer: calls that overlap on one
 * device (concurrent streams, or threads) race and must be ordered by the
 * caller.  Without a split (ksplit 1, or K <= 64) no scratch is used. */
int tp_minplus_gemm_ex_noalloc(int dtype, int64_t M, int64_t N, int64_t K, const void *d_A,
                               int64_t lda, const void *d_B, int64_t ldb, void *d_C,
                               int64_t ldc, int accumulate, int config, int ksplit,
                               hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Tuning tables (filled by the autotuner; the library has built-in          */
/* defaults).  None of them changes a result, only which kernel shape runs.  */
/* ------------------------------------------------------------------------ */

/* Default product shape: tp_minplus_gemm (and every dense product the
 * library runs itself) uses, for max(M, N, K) <= max_dim, the entry with the
 * smallest such max_dim: tile configuration `config` and K split `ksplit`.
 * Setting an existing max_dim replaces it; max_dim < 0 clears the dtype's
 * table (back to the built-in heuristic).  Process-wide, thread-safe. */
int tp_tune_gemm(int dtype, int64_t max_dim, int config, int ksplit);

/* The tuned (config, ksplit) for an M x N x K product of this dtype, into
 * *config and *ksplit (host pointers): the shape of the library's own
 * products; tp_minplus_gemm runs that config with ksplit 1. */
int tp_gemm_choice(int dtype, int64_t M, int64_t N, int64_t K, int *config, int *ksplit);

/* Measured rates for the schedule planner of tp_tropical_power_trace at path
 * order n (1..12): (min,+) operations per second of one sparse left step
 * (nnz * N operations) and of one dense product (N^3).  Positive values, or
 * both 0 to restore the built-in rates. */
int tp_tune_planner(int n, double spmm_ops_per_s, double gemm_ops_per_s);

/* Library-wide defaults of the batch engine's baby steps c at path order n
 * (1..12), for the default mode and for TP_PARAM_FUSED_CHAIN (where the
 * levels of all n of a batch run together); 0 keeps the built-in rule.  A
 * context's TP_PARAM_BABY_STEPS takes precedence; baby steps already fixed in
 * a context do not change.  A set created from these defaults (16-bit powers,
 * giants by products) takes c = ceil(m_max / 2) instead, m_max the largest
 * cycle order of n in the batch that creates it, when some instance needs a
 * giant at c and either that is at most 2c and tp_tune_planner's rates put
 * the extra chain levels below the giants' products, or (fused mode) it is
 * within the batch's deepest chain of levels, which run anyway. */
int tp_tune_batch(int n, int baby_steps, int fused_baby_steps);

/* Matrix-vector products with the M x K matrix A:
 *   trans == 0:  y (M)  = A x x (x has K entries),  y_i = min_k a_ik + x_k
 *   trans == 1:  y (K)  = x x A (x has M entries),  y_k = min_i x_i + a_ik
 * Device pointers of the given dtype. */
int tp_minplus_gemv(int dtype, int64_t M, int64_t K, const void *d_A, int64_t lda,
                    const void *d_x, void *d_y, int trans, hipStream_t stream);

/* Y (rows x ncols) = S x X where S is the sparse rows x K matrix with
 * S[q][p] = d_z[p] for p in d_col[d_rowptr[q] .. d_rowptr[q+1]-1] and INF
 * elsewhere (the shape of A(D_n) from tp_build_state_csr, whose labels depend
 * on the column only), and X is dense K x ncols.  One left multiplication of
 * the power chain of Algorithm 2 costs nnz * ncols (min,+) operations this
 * way.  Column indices must be < K; K is only used for that check. */
int tp_minplus_spmm(int dtype, int64_t rows, int64_t K, const int64_t *d_rowptr,
                    const uint32_t *d_col, const uint8_t *d_z, const void *d_X, int64_t ldx,
                    void *d_Y, int64_t ldy, int64_t ncols, hipStream_t stream);

/* Forms of the sparse left step by the state matrix. */
#define TP_STEP_AUTO 0    /* the tuned (or built-in) choice for n */
#define TP_STEP_CSR 1     /* one wave per row gathering its successors' rows */
#define TP_STEP_BLOCKED 2 /* the union of the successor lists of 16
                           * consecutive rows, walked once per block a run of
                           * successors shared by the same rows at a time (one
                           * minimum per run, then applied to those rows), so
                           * each gathered row of X is read once per block */
#define TP_STEP_BLOCKED_ENTRIES 3 /* the same union, each successor applied
                                   * to its rows on its own */

/* Y (N x ncols, u16) = A(D_n) x X (X: N x ncols, u16), N = tp_state_dim(n):
 * the left multiplication of Algorithm 2's power chain by the state matrix
 * itself, with the library's resident forms of A(D_n) (built and cached on
 * first use per device and n).  Every form gives the result of
 * tp_minplus_spmm with the CSR of tp_build_state_csr; TP_STEP_AUTO takes
 * the form tp_tune_step set for n, else row blocks from n = 11 on (measured
 * faster there) and the CSR gather below.  X and Y must not overlap.
 * Leading dimensions in elements; 1 <= n <= 13.  TP_EINVAL on a bad n, form
 * or size. */
int tp_state_left_mul(int n, int form, const void *d_X, int64_t ldx, void *d_Y, int64_t ldy,
                      int64_t ncols, hipStream_t stream);

/* The form TP_STEP_AUTO uses at path order n (TP_STEP_AUTO: the built-in
 * rule).  The power chains of tp_tropical_power_trace use it too. */
int tp_tune_step(int n, int form);

/* Compact powers: a power P of A(D_n) held as 8-bit residuals x plus one
 * int32 offset per row, P[q][c] = R[q] + x[q][c] with x in 0..254; a row of
 * INF entries only is R[q] = 0x3FFFFFFF with x = 255.  Half the bytes of the
 * 16-bit form for the power chain of Algorithm 2.  Status words are device
 * int32 that the calls OR bits into (the caller clears them and reads them
 * when convenient): 1 = a row spans more than 254 or a result cannot be held
 * (the matrix written is then not valid), 2 = a row mixes finite and INF
 * entries (the same).  Leading dimensions are in elements (bytes for the
 * residuals). */

/* d_Y (N x ncols, u8 residuals) and d_R (N, int32) from the 16-bit matrix
 * d_X (N x ncols): R[q] = least entry of row q, x = entry - R[q].  One
 * workgroup per row.  TP_EINVAL on a bad size or NULL pointer. */
int tp_compact_from_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx, void *d_Y,
                        int64_t ldy, int32_t *d_R, int32_t *d_status, hipStream_t stream);

/* d_Y (N x ncols, u16) = min(R[q] + x[q][c], INF = 65535), x = 255 giving
 * INF: the 16-bit form of a compact power, equal to the 16-bit chain's. */
int tp_compact_to_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx, const int32_t *d_R,
                      void *d_Y, int64_t ldy, hipStream_t stream);

/* (d_Y, d_RY) = A(D_n) x (d_X, d_RX) in compact form, N = tp_state_dim(n)
 * rows of ncols columns: Algorithm 2's left step with the arc labels of
 * Section 2.2 (they depend on the successor only, so a row's new offset is
 * min over its successors p of z_p + R_X[p] and the residuals need one add
 * per gathered row).  The residuals of a held power never grow under the
 * step, so a held input gives a held output.  d_X and d_Y: 8-byte aligned,
 * ld a multiple of 8 and at least ncols rounded up to 8; X, Y and the two
 * offset vectors must not overlap.  1 <= n <= 13.  Uses the cached blocked
 * and CSR forms of A(D_n) (built on first use per device and n). */
int tp_compact_step(int n, const void *d_X, int64_t ldx, const int32_t *d_RX, void *d_Y,
                    int64_t ldy, int32_t *d_RY, int64_t ncols, int32_t *d_status,
                    hipStream_t stream);

/* *d_out = min over rows q with x[q][q] != 255 of min(R[q] + x[q][q], 65535)
 * (65535 when there is none): the diagonal minimum of Theorem 2 on a square
 * compact power (ldx >= N). */
int tp_compact_diag_min(int64_t N, const void *d_X, int64_t ldx, const int32_t *d_R,
                        int32_t *d_out, hipStream_t stream);

/* Shared-base compact powers: one base G per power, P[q][c] = G + x[q][c]
 * with x in 0..254 and every entry finite; d_base is a device int32[2]
 * holding G and the least residual held.  A whole power of A(D_n) spans a
 * few units more than one of its rows, so it fits too, and the step adds
 * only the arc label per gathered row (no per-row offset).  Status bits as
 * above. */

/* d_Y (u8 residuals) and d_base from the 16-bit d_X: G = least entry;
 * an INF entry sets status bit 2, a residual above 254 bit 1. */
int tp_compact_shared_from_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx,
                               void *d_Y, int64_t ldy, int32_t *d_base, int32_t *d_status,
                               hipStream_t stream);

/* d_Y (u16) = min(G + x, INF = 65535). */
int tp_compact_shared_to_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx,
                             const int32_t *d_base, void *d_Y, int64_t ldy, hipStream_t stream);

/* (d_Y, d_by) = A(D_n) x (d_X, d_bx), Algorithm 2's left step: the output is
 * held over G_Y = G_X + (least residual of X), which no entry of the output
 * is below (labels are non-negative), so its residuals are its span plus the
 * growth of its least entry; one above 254 sets status bit 1.  Layout
 * requirements as tp_compact_step; d_bx and d_by distinct. */
int tp_compact_shared_step(int n, const void *d_X, int64_t ldx, const int32_t *d_bx, void *d_Y,
                           int64_t ldy, int32_t *d_by, int64_t ncols, int32_t *d_status,
                           hipStream_t stream);

/* *d_out = min(min over q of G + x[q][q], 65535): Theorem 2's diagonal
 * minimum of a square shared-base power. */
int tp_compact_shared_diag_min(int64_t N, const void *d_X, int64_t ldx, const int32_t *d_base,
                               int32_t *d_out, hipStream_t stream);

/* *d_out = min(65535, G_X + G_P + min over t < count and k < N of
 * x[r_t][k] + p[k][t]), r_t = d_idx[t] (r_t = t when d_idx is NULL, which
 * needs count <= N): Theorem 2's trace of the product X x P read only on the
 * diagonal entries of the listed states, for X a square shared-base power
 * (N x N, rows r_t read) and P an N x count shared-base panel whose column t
 * belongs to state r_t (the columns d_idx of another power, as
 * tp_build_state_columns lays them out).  With d_idx NULL and count = N it is
 * the whole trace of the product, min_i (X x P)_ii.  d_bx, d_bp: the two
 * base words (G first).  Every d_idx[t] must lie in 0..N-1 (device memory,
 * not checked).  16-byte aligned rows with ld a multiple of 16 take the
 * vector path; any layout with ldx >= N, ldp >= count is accepted. */
int tp_compact_shared_select_trace(int64_t N, int64_t count, const int32_t *d_idx,
                                   const void *d_X, int64_t ldx, const int32_t *d_bx,
                                   const void *d_P, int64_t ldp, const int32_t *d_bp,
                                   int32_t *d_out, hipStream_t stream);

/* Gathers per round in tp_compact_step and tp_compact_shared_step (4 or 8),
 * optionally | TP_COMPACT_GROUPED: the shared-base step then takes each row
 * block's successors a mask group at a time (one minimum per run of
 * successors shared by the same rows, then applied to those rows).  0
 * restores the default, 4 | TP_COMPACT_GROUPED.  Changes speed only. */
#define TP_COMPACT_GROUPED 0x100
int tp_tune_compact_step(int unroll);

/* All-pairs shortest paths by (min,+) squaring, the same semiring (Section 1)
 * on another workload: d_D (N x N) = (I + W)^(2^t), t = ceil(log2(N - 1)),
 * where W holds non-negative arc weights (INF = no arc) and I is the (min,+)
 * identity, so d_D[i][j] = min(least weight of a path i -> j, INF) exactly
 * (sums saturate; with non-negative weights the saturated sum of a path does
 * not depend on the order of its additions).  d_T is an N x N work matrix
 * (ldt >= N), distinct from d_W and d_D, unused when N <= 2; d_W may be
 * d_D.  t dense products of N^3 operations each; no allocation. */
int tp_apsp(int dtype, int64_t N, const void *d_W, int64_t ldw, void *d_D, int64_t ldd,
            void *d_T, int64_t ldt, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Traces: Theorem 2 reads gamma_2 as the minimum of the diagonal.            */
/* ------------------------------------------------------------------------ */

/* *d_out (device int32) = min_i X_ii over the N x N matrix X (INF if N = 0). */
int tp_trace_min(int dtype, int64_t N, const void *d_X, int64_t ldx, int32_t *d_out,
                 hipStream_t stream);

/* *d_out = min_i (X x Y)_ii = min_{i,k} x_ik + y_ki for N x N matrices, without
 * forming the product; saturates at the dtype's INF. */
int tp_trace_of_product(int dtype, int64_t N, const void *d_X, int64_t ldx, const void *d_Y,
                        int64_t ldy, int32_t *d_out, hipStream_t stream);

/* *d_out = min over arcs q -> p of d_z[p] + X[p][q]: the trace of S x X for the
 * sparse S of tp_minplus_spmm with rows = K = N. */
int tp_sparse_trace_of_product(int dtype, int64_t N, const int64_t *d_rowptr,
                               const uint32_t *d_col, const uint8_t *d_z, const void *d_X,
                               int64_t ldx, int32_t *d_out, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* gamma_2(P_n x C_m) = min_i (A(D_n)^m)_ii (Theorem 2).                       */
/* ------------------------------------------------------------------------ */

/* Computes gamma_2(P_n x C_m) for 1 <= n <= 12, m >= 3 into *gamma2_host and
 * blocks until it is known.  The schedule (chain of sparse left products,
 * dense squarings, a final trace of a product) is chosen by a cost model; the
 * result does not depend on it.  State matrices and work buffers are kept in
 * a process-wide cache on the current device (grown on demand; freed by
 * tp_release_cache).  TP_EOVERFLOW when n*m >= 65535. */
int tp_tropical_power_trace(int n, int64_t m, int32_t *gamma2_host, hipStream_t stream);

/* Frees the process-wide cache used by tp_tropical_power_trace. */
int tp_release_cache(void);

/* Start states pruned by the cycle's rotation symmetry.  A closed walk of
 * length m visits m states whose zero counts add up to its label (Theorem 2),
 * so an optimal walk passes through a state with at most floor(gamma_2 / m)
 * zeros and may start there: gamma_2 = min over the states i with at most
 * floor(gamma_2 / m) zeros of (A^m)_ii, computed from the columns i of the
 * powers only.  tp_tropical_power_trace uses it when its cost model says so
 * (first with a guessed bound k, then, if the value found allows more zeros,
 * once more with floor(value / m)). */

/* Indices (ascending, int32) of the states of A(D_n) with at most max_zeros
 * zeros, into d_idx (device, room for cap; may be NULL to count only), queued
 * on `stream`.  Returns the count or a negative status. */
int64_t tp_state_select(int n, int max_zeros, int32_t *d_idx, int64_t cap, hipStream_t stream);

/* d_X (u16, N x count, leading dimension ldx >= count, N = tp_state_dim(n))
 * = the columns d_idx[0..count) of A(D_n); an index outside 0..N-1 gives a
 * column of INF. */
int tp_build_state_columns(int n, const int32_t *d_idx, int64_t count, void *d_X, int64_t ldx,
                           hipStream_t stream);

/* *d_out (device int32) = min_j d_X[d_idx[j]][j] over j < count whose index
 * lies in 0..N-1 (u16 X with N rows, ldx >= count); INF when there is none. */
int tp_diag_select_min(int64_t N, int64_t count, const int32_t *d_idx, const void *d_X,
                       int64_t ldx, int32_t *d_out, hipStream_t stream);

/* How tp_tropical_power_trace uses pruned start states: 0 = when its cost
 * model prefers it (default), 1 = always, -1 = never.  Changes no result. */
int tp_tune_prune(int mode);

/* ------------------------------------------------------------------------ */
/* Recurrence of the powers: Lemma 1, Theorem 3, Algorithms 3, 4 and 5.      */
/* ------------------------------------------------------------------------ */

/* Matrix constant difference (Algorithm 3's test, exact reading): X and Y
 * (u16, N x N) differ by a constant when they have the same INF entries and
 * every finite entry of X is the matching entry of Y plus one common b, i.e.
 * X = b (x) Y.  d_out (device int32[2]) receives {min, max} of the finite
 * differences X - Y: min == max == b when it holds; min > max (INT32_MAX,
 * INT32_MIN) when no entry is finite (it holds with b = 0); min < max when it
 * fails (INF patterns that differ count as -2^30 and 2^30).  Needs ldx == ldy,
 * a multiple of 8, and 16-byte aligned X and Y.  Reads 2 N^2 entries once
 * (HBM bound); its small work buffer is stream-ordered (hipMallocAsync). */
int tp_const_diff(int64_t N, const void *d_X, int64_t ldx, const void *d_Y, int64_t ldy,
                  int32_t *d_out, hipStream_t stream);

/* Result of tp_recurrence (all exponents are powers of A = A(D_n)). */
typedef struct tp_recurrence {
  int32_t found;        /* 1: A^(r0 + a) = b (x) A^r0 among A^1 .. A^K               */
  int32_t window_short; /* 1: not found, and pairs Algorithm 3 would examine before
                           giving up lay beyond the window                           */
  int32_t K;            /* powers computed                                           */
  int32_t window;       /* each A^k was compared with A^(k-1) .. A^(k-window)         */
  int64_t r0, a, b;     /* Algorithm 3: the first pair (i, j) = (r0 + a, r0), i from K
                           down, j from i - 1 down, with A^i = b (x) A^j (Table 3)    */
  int64_t n0;           /* Algorithm 4: least n0 such that A^(k + a) = b (x) A^k for
                           n0 <= k <= r0, going down from r0 (Table 4)               */
} tp_recurrence_t;

/* Computes A^1 .. A^K of A(D_n) (1 <= n <= 13) by the chain of sparse left
 * products (Algorithm 2), keeping only the last window + 1 powers on the
 * device; compares each A^k with A^(k-d), 1 <= d <= min(window, k - 1), by
 * tp_const_diff, and writes diag_min_host[k - 1] = min_i (A^k)_ii for
 * k = 1..K (host int32[K]; Algorithm 5's boundary values, gamma_2(P_n x C_k)
 * for k >= 3 by Theorem 2).  Then runs Algorithms 3 and 4 on the comparison
 * table into *out.  Algorithm 3's result equals the paper's exactly when it is
 * found at i = K (every smaller distance was compared) or when window =
 * K - 1 (every pair was); otherwise found = 0 and window_short = 1.
 * 2 <= K <= 65535; 0 <= window <= 256, where 0 picks min(K - 1, 256) when
 * those powers fit in free device memory, else the most that fit.  Device
 * memory: (window + 1) N x round64(N) u16 powers, allocated and freed by the
 * call, plus the state of n (process-wide cache).  Blocks until done.
 * TP_EOVERFLOW when n * K >= 65535; TP_ENOMEM when an explicit window does
 * not fit. */
int tp_recurrence(int n, int K, int window, tp_recurrence_t *out, int32_t *diag_min_host,
                  hipStream_t stream);

/* Path orders from which the power chains of tp_recurrence and of
 * tp_tropical_power_trace's pruned plans run on shared-base compact powers
 * (u8 residuals over one base per power, from the first power with no INF
 * entry on): 11 by default, where that step is faster than the 16-bit one;
 * 0 keeps every chain in 16 bits.  Results are the same either way: in the
 * recurrence, powers before the switch hold INF entries, so their
 * comparisons with the all-finite later ones fail as in 16 bits; a power
 * that cannot be held sends the call back to the 16-bit chain. */
int tp_tune_compact_chains(int compact_from_n);

/* gamma_2(P_n x C_m) for any m >= 3 from a recurrence and its boundary values
 * (host only, no device work): diag_min[m - 1] when m <= K, else, when the
 * recurrence was found, Theorem 3's finite difference equation solved from
 * its start: gamma_2(n0 + r + q a) = gamma_2(n0 + r) + q b with 0 <= r < a.
 * TP_EINVAL for m < 3, or m > K without a recurrence. */
int tp_gamma2_recurrence(const tp_recurrence_t *rec, const int32_t *diag_min, int64_t m,
                         int64_t *gamma2);

/* ------------------------------------------------------------------------ */
/* Batching: many (n, m) instances per call, one persistent launch each.     */
/* ------------------------------------------------------------------------ */

/* A context keeps powers of A = A(D_n) resident in device memory (u16, rows
 * padded to 64 entries), at most hbm_budget_bytes in total: per n the chain
 * A^1..A^c of Algorithm 2 and giants A^(jc) formed by dense products of
 * resident powers.  gamma_2(P_n x C_m) is the trace of A^a x A^b for a + b = m
 * (Theorem 2): (ceil(m/2), floor(m/2)) when m <= 2c, else (jc, m - jc) with
 * 1 <= m - jc <= c.  Path orders from TP_PARAM_COMPACT_FROM on (default 10)
 * keep A^3 and every higher power as shared-base compact powers instead (u8
 * residuals over one base per power, half the bytes; A^1 .. A^3 also in 16
 * bits): babies run to c + 2 (c >= 4), and a pair with an exponent above 3
 * has both at 3 or above: (ceil(m/2), floor(m/2)) when m <= 2(c + 2), else
 * (jc, m - jc) with 3 <= m - jc <= c + 2; a giant is the product of two
 * compact powers (residuals summed in 16 bits, bases added), a trace adds the
 * two bases to the residuals' minimum.  From TP_PARAM_CHAIN_GIANTS_FROM on
 * (default 10) the giants come from the chain itself instead.  Powers persist
 * across batches until the context is destroyed.  A context is used from one
 * host thread and one stream at a time. */
int tp_ctx_create(size_t hbm_budget_bytes, void **ctx);
int tp_ctx_destroy(void *ctx);

/* Tuning and test parameters of a context. */
#define TP_PARAM_WAIT_LIMIT_US 1 /* bound on one dependency wait (default 20 s) */
#define TP_PARAM_GRID 2          /* workgroups of the persistent kernel (>= 8); 0 = fill the chip */
#define TP_PARAM_FUSED_CHAIN 3   /* 1: chain levels run inside the persistent launch too (one
                                    launch per batch, levels separated by barriers over the
                                    grid, which then never exceeds what the chip holds);
                                    0 (default): as full-chip launches on one stream per n
                                    ahead of it */
#define TP_PARAM_COMPACT_FROM 4  /* path orders n >= value keep compact powers from A^3 on
                                    (0: none; default 10); fixed per n once its powers are
                                    resident.  A batch with compact sets runs their chain
                                    levels as launches in either mode */
#define TP_PARAM_CHAIN_GIANTS_FROM 5 /* path orders n >= value make their giants by continuing
                                    the chain (sparse left steps through two more buffers of
                                    the set, no smaller giants) instead of dense products
                                    (0: never; default 10, where jc steps cost less than the
                                    products); fixed per n once its powers are resident */
#define TP_PARAM_BABY_STEPS 32   /* TP_PARAM_BABY_STEPS + n: chain length c; 0 = auto (16 for
                                    n >= 8, else 32); fixed once powers of n are resident */
int tp_ctx_set_param(void *ctx, int param, int64_t value);

/* Bytes of resident powers held by the context. */
int64_t tp_ctx_resident_bytes(void *ctx);

/* Frees the resident powers of path order n (n = 0: of every n), after
 * waiting for the work queued on `stream`. */
int tp_ctx_release(void *ctx, int n, hipStream_t stream);

/* Copies the resident power A(D_n)^e of a context (Section 2.2's state
 * matrix raised in the (min,+) semiring, as the context's batches computed
 * it) into d_out: device u16, N rows padded to ld >= N entries, N =
 * tp_state_dim(n); on `stream`, after the work queued there (a batch that
 * computes the power must be queued on the same stream or finished).
 * TP_EINVAL when the context holds no such power or ld < N.  The caller owns
 * d_out. */
int tp_ctx_copy_power(void *ctx, int n, int e, void *d_out, int64_t ld, hipStream_t stream);

/* Bytes of powers a batch of these instances would add to the context (0
 * when everything it needs is resident); for admission control.  Host
 * planning only, except that a new set whose baby steps come from
 * tp_tune_batch's defaults and whose choice needs the planner's cost builds
 * the state of n (once per process, as the batch would). */
int64_t tp_ctx_need_bytes(void *ctx, int count, const int32_t *n, const int64_t *m);

/* gamma2_dev[j] (device int32) = gamma_2(P_{n[j]} x C_{m[j]}) for j < count,
 * with n (host int32) in 1..12 and m (host int64) >= 3, n*m < 65535.  Queues
 * the missing chain levels of every distinct n (A^1 and the sparse left
 * steps, one context-owned stream per n, ordered after the work already on
 * `stream`), then, on `stream`, the missing giant products and one trace per
 * instance as one dependency-ordered task list run by one persistent kernel
 * launch from a captured hipGraph; with TP_PARAM_FUSED_CHAIN the chain levels
 * run first inside that one launch, level by level with a barrier over the
 * grid between levels.  Returns without waiting.
 * TP_ENOMEM when the needed powers exceed the context's budget (nothing is
 * queued).  Results of a batch are valid after tp_ctx_check returns TP_OK. */
int tp_batch_power_trace(void *ctx, int count, const int32_t *n, const int64_t *m,
                         int32_t *gamma2_dev, hipStream_t stream);

/* The algorithmic work of the last batch queued on ctx, for roofline
 * accounting: ops[0] = (min,+) operations of its chain levels (nnz(A(D_n)) * N
 * per level computed), ops[1] = of its dense giant products (N^3 each),
 * ops[2] = of its traces of products (N^2 per instance); *bytes = the bytes
 * those must move at the least with 16-bit entries (4 N^2 per level, 6 N^2
 * per product, 4 N^2 per trace, 2 N^2 for A^1).  Work that resident powers
 * made unnecessary is not counted.  Host pointers; no GPU work. */
int tp_ctx_last_work(void *ctx, double *ops, double *bytes);

/* Waits for `stream` and reports whether the batches queued since the last
 * check completed: TP_OK, or TP_ECANCELED when a task's wait for its inputs
 * exceeded the wait limit (the kernel then drains without computing, the
 * results are invalid and the levels it was to compute are dropped), or
 * TP_EOVERFLOW when a compact power would have needed a residual above 254
 * (results invalid, its powers dropped; for the powers of A(D_n) the
 * residuals stay within a few units of n). */
int tp_ctx_check(void *ctx, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Small cycle, any path.  Section 1 names the complementary problem (a       */
/* small cycle and a path of any order, by (min,+) matrix-vector products);   */
/* Section 2.1's column digraph applies with columns that are copies of the   */
/* cycle C_m, the rules of Section 2.2 read around the cycle (letter i's      */
/* column neighbours are i - 1 and i + 1 modulo m), and an open walk of n     */
/* columns along the path.  The first column is labelled from its own column  */
/* (no column before it); the last holds no 2 (no column after it gives a 2   */
/* its second neighbour).  Then                                               */
/*   gamma_2(P_n x C_m) = min_p (start x A^(n-1))_p + end_p,                  */
/* start_p = zeros(p) where p may open the walk (else INF), end_p = 0 where   */
/* p may close it (else INF), A[q][p] = zeros(p) if p can follow q, else INF. */
/* Cyclic words are indexed in increasing base-3 value (first letter most     */
/* significant).  3 <= m <= 12 (N < 65536); TP_EINVAL otherwise.              */
/* ------------------------------------------------------------------------ */

/* Number of correct cyclic words of length m (host count, no GPU work). */
int64_t tp_cyclic_dim(int m);

/* Number of arcs (non-INF entries of A); the first call for m builds the
 * cyclic digraph on the current device and blocks; later calls are cached. */
int64_t tp_cyclic_nnz(int m);

/* d_codes[0..N-1] = base-3 codes of the correct cyclic words, increasing
 * (device uint32_t array of N = tp_cyclic_dim(m) entries). */
int tp_cyclic_words(int m, uint32_t *d_codes, hipStream_t stream);

/* The N x N matrix A of the cyclic column digraph, dtype TP_U8 or TP_U16,
 * row-major with leading dimension lda >= N (device memory of the caller). */
int tp_build_cyclic_matrix(int m, int dtype, void *d_A, int64_t lda, hipStream_t stream);

/* The walk's boundary vectors (N entries each, dtype TP_U8 or TP_U16):
 * d_start[p] = zeros(p) if p may be the first column else INF; d_end[p] = 0
 * if p may be the last column else INF.  Either pointer may be NULL (that
 * vector is not written), not both. */
int tp_build_cyclic_boundary(int m, int dtype, void *d_start, void *d_end, hipStream_t stream);

/* gamma_2(P_n x C_m) into *gamma2_host for n >= 1, blocking: the walk as
 * n - 1 dense vector-matrix products x <- x x A (the kernel of
 * tp_minplus_gemv with trans = 1, on a cached u16 copy of A) and the end
 * vector.  TP_EOVERFLOW when n*m >= 65535.  The cache (digraph, dense A,
 * level vectors) lives on the current device until tp_release_cache. */
int tp_cyclic_walk_gamma2(int64_t n, int m, int32_t *gamma2_host, hipStream_t stream);

/* Forms of the sweep below; every form gives the same numbers. */
#define TP_WALK_AUTO 0  /* the one-workgroup walk where it fits, else TP_WALK_STEPS */
#define TP_WALK_CHAIN 1 /* the whole walk in one launch of one workgroup, level
                         * vectors in LDS (N <= 10752, m <= 10) */
#define TP_WALK_STEPS 2 /* one full-chip launch per level: a wave per column
                         * gathers the minimum over its predecessors */
#define TP_WALK_GEMV 3  /* one dense vector-matrix product per level */

/* d_gamma2[k - 1] (device int32) = gamma_2(P_k x C_m) for k = 1..nmax: one
 * walk whose every level is read by the end vector.  TP_WALK_CHAIN returns
 * without waiting; the other forms use the cache's level vectors and block
 * until done.  TP_EOVERFLOW when nmax*m >= 65535; TP_EINVAL when
 * TP_WALK_CHAIN is asked for an m whose words do not fit. */
int tp_cyclic_walk_sweep(int m, int64_t nmax, int32_t *d_gamma2, int form, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TROPICAL_H */
