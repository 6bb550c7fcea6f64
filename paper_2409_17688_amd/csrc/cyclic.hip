// Small cycle, any path: columns that are copies of the cycle C_m and an open
// walk of n columns along the path P_n.  Section 1 names this complementary
// problem (solved in the companion work with (min,+) matrix-vector
// products); Section 2.1 gives the column digraph for any Cartesian product
// with a column structure, and the letters and rules of Section 2.2 carry
// over with the neighbours of letter i inside a column taken around the
// cycle (letters i - 1 and i + 1 modulo m).
//
// Words.  A cyclic word is correct when none of its m windows of three
// letters, read around the cycle, is 020 or has a 1 between two non-zero
// letters.  A word's rank among the correct ones comes from a completion
// table indexed by its first two letters (the two windows that close the
// cycle need them) and its last two, so each thread ranks its own code.
//
// Arcs.  Masks as for the path words (bit i = letter i is 0, bit 16 + i =
// letter i is 1); the rotation by one position replaces the shift, so the
// follow test stays a few bitwise operations.  The first column of the walk
// follows an absent column (no 0, no 2): its letters are labelled from their
// own column.  The last column has no column after it to give a 2 its second
// neighbour, so it holds no 2.
//
// The walk's labels: x_1 = start, x_(k+1) = x_k x A, and
// gamma_2(P_k x C_m) = min_p x_k[p] + end[p].  With the arc label depending on
// the successor only, (x x A)_p = z_p + min over the predecessors q of p of
// x_q, so a step is a gather-min over predecessor lists (kept as a CSR of
// the columns of A, 16-bit indices: N < 65536 for m <= 12) and one add.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace tp {

namespace {

constexpr int kMaxM = 12;

__host__ __device__ inline bool cyc_window_ok(int a, int b, int c) {
  if (a == 0 && b == 2 && c == 0) return false;  // 020
  if (b == 1 && a != 0 && c != 0) return false;  // a 1 between two non-zero letters
  return true;
}

// g[r][h][t]: ways to append r letters after a prefix whose first two
// letters are h = (c0, c1) and last two t = (a, b), such that every new
// window and the two windows around the end of the cycle hold.
__host__ __device__ inline void build_cyclic_completions(int m, int32_t (*g)[9][9]) {
  for (int h = 0; h < 9; ++h)
    for (int t = 0; t < 9; ++t) {
      const int c0 = h / 3, c1 = h % 3, a = t / 3, b = t % 3;
      g[0][h][t] = (cyc_window_ok(a, b, c0) && cyc_window_ok(b, c0, c1)) ? 1 : 0;
    }
  for (int r = 1; r <= m - 2; ++r)
    for (int h = 0; h < 9; ++h)
      for (int t = 0; t < 9; ++t) {
        const int a = t / 3, b = t % 3;
        int32_t s = 0;
        for (int c = 0; c < 3; ++c)
          if (cyc_window_ok(a, b, c)) s += g[r - 1][h][b * 3 + c];
        g[r][h][t] = s;
      }
}

__global__ void cyclic_words_kernel(int m, uint32_t total, uint32_t *__restrict__ codes,
                                    uint8_t *__restrict__ zeros, uint32_t *__restrict__ masks) {
  __shared__ int32_t g[kMaxM - 1][9][9];
  if (threadIdx.x == 0) build_cyclic_completions(m, g);
  __syncthreads();
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total) return;
  int w[kMaxM];
  uint32_t t = x;
  for (int i = m - 1; i >= 0; --i) {
    w[i] = (int)(t % 3u);
    t /= 3u;
  }
  for (int i = 0; i < m; ++i)
    if (!cyc_window_ok(w[(i + m - 1) % m], w[i], w[(i + 1) % m])) return;
  // rank = number of correct cyclic words below x
  int64_t rank = 0;
  for (int c = 0; c < w[0]; ++c)
    for (int d = 0; d < 3; ++d) rank += g[m - 2][c * 3 + d][c * 3 + d];
  for (int d = 0; d < w[1]; ++d) rank += g[m - 2][w[0] * 3 + d][w[0] * 3 + d];
  const int h = w[0] * 3 + w[1];
  for (int i = 2; i < m; ++i)
    for (int c = 0; c < w[i]; ++c)
      if (cyc_window_ok(w[i - 2], w[i - 1], c)) rank += g[m - 1 - i][h][w[i - 1] * 3 + c];
  uint32_t zm = 0, om = 0;
  for (int i = 0; i < m; ++i) {
    zm |= (w[i] == 0 ? 1u : 0u) << i;
    om |= (w[i] == 1 ? 1u : 0u) << i;
  }
  if (codes) codes[rank] = x;
  if (zeros) zeros[rank] = (uint8_t)__builtin_popcount(zm);
  if (masks) masks[rank] = zm | (om << 16);
}

// Zeros of the column neighbours around the cycle: bit i of prev is letter
// i - 1, bit i of next is letter i + 1 (indices modulo m).
__device__ __forceinline__ uint32_t cyc_prev(uint32_t z, int m, uint32_t full) {
  return ((z << 1) | (z >> (m - 1))) & full;
}
__device__ __forceinline__ uint32_t cyc_next(uint32_t z, int m) {
  return (z >> 1) | ((z & 1u) << (m - 1));
}

// p can follow q: every 2 of q over a 0 of p; every 2 of p sees exactly one
// 0 among q_i and its two column neighbours; every 1 of p at least two.
__device__ __forceinline__ bool cyc_follows(uint32_t mq, uint32_t mp, int m, uint32_t full) {
  const uint32_t zq = mq & 0xFFFFu, oq = mq >> 16, tq = full & ~(zq | oq);
  const uint32_t zp = mp & 0xFFFFu, op = mp >> 16, tp = full & ~(zp | op);
  const uint32_t x = zq, y = cyc_prev(zp, m, full), w = cyc_next(zp, m);
  const uint32_t exactly_one = (x ^ y ^ w) & ~(x & y & w);
  const uint32_t two_or_more = (x & y) | (x & w) | (y & w);
  return ((tq & ~zp) | (tp & ~exactly_one) | (op & ~two_or_more)) == 0;
}

// The first column: the same rules after a column with no 0 and no 2.
__device__ __forceinline__ bool cyc_can_start(uint32_t mp, int m, uint32_t full) {
  const uint32_t zp = mp & 0xFFFFu, op = mp >> 16, tp = full & ~(zp | op);
  const uint32_t y = cyc_prev(zp, m, full), w = cyc_next(zp, m);
  return ((tp & ~(y ^ w)) | (op & ~(y & w))) == 0;
}

// The last column: no 2.
__device__ __forceinline__ bool cyc_can_end(uint32_t mp, uint32_t full) {
  return (full & ~((mp & 0xFFFFu) | (mp >> 16))) == 0;
}

template <typename T, T INF>
__global__ void cyclic_dense_kernel(int m, int64_t N, const uint32_t *__restrict__ masks,
                                    T *__restrict__ A, int64_t lda) {
  const uint32_t full = (1u << m) - 1u;
  const int64_t q = blockIdx.x;
  const uint32_t mq = masks[q];
  T *row = A + q * lda;
  for (int64_t p = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.y * blockDim.x) {
    const uint32_t mp = masks[p];
    row[p] = cyc_follows(mq, mp, m, full) ? (T)__builtin_popcount(mp & 0xFFFFu) : INF;
  }
}

template <typename T, T INF>
__global__ void cyclic_boundary_kernel(int m, int64_t N, const uint32_t *__restrict__ masks,
                                       T *__restrict__ start, T *__restrict__ end) {
  const uint32_t full = (1u << m) - 1u;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t mp = masks[p];
  if (start) start[p] = cyc_can_start(mp, m, full) ? (T)__builtin_popcount(mp & 0xFFFFu) : INF;
  if (end) end[p] = cyc_can_end(mp, full) ? (T)0 : INF;
}

// One wave per column p: its in-degree into predptr[p + 1].
__global__ void cyclic_pred_count_kernel(int m, int64_t N, const uint32_t *__restrict__ masks,
                                         int64_t *__restrict__ predptr) {
  const uint32_t full = (1u << m) - 1u;
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (p >= N) return;
  const uint32_t mp = masks[p];
  int64_t cnt = 0;
  for (int64_t q0 = 0; q0 < N; q0 += 64) {
    const int64_t q = q0 + lane;
    const bool arc = q < N && cyc_follows(masks[q], mp, m, full);
    cnt += __popcll(__ballot(arc));
  }
  if (lane == 0) {
    predptr[p + 1] = cnt;
    if (p == 0) predptr[0] = 0;
  }
}

// One wave per column p: its predecessors in increasing order.
__global__ void cyclic_pred_fill_kernel(int m, int64_t N, const uint32_t *__restrict__ masks,
                                        const int64_t *__restrict__ predptr,
                                        uint16_t *__restrict__ pred) {
  const uint32_t full = (1u << m) - 1u;
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (p >= N) return;
  const uint32_t mp = masks[p];
  int64_t pos = predptr[p];
  for (int64_t q0 = 0; q0 < N; q0 += 64) {
    const int64_t q = q0 + lane;
    const bool arc = q < N && cyc_follows(masks[q], mp, m, full);
    const uint64_t b = __ballot(arc);
    if (arc) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      pred[pos + below] = (uint16_t)q;
    }
    pos += __popcll(b);
  }
}

// Per-thread strips for the one-workgroup chain: the predecessor list,
// concatenated in column order, is cut into strips of `per` consecutive
// entries, strip t for thread t; entry i of strip t sits at i * threads + t,
// so the threads' loads of one round are adjacent.  An entry packs the
// column p (high 16 bits) and the predecessor q (low 16 bits); padding is
// 0xFFFFFFFF.  One wave per column p writes its entries.
__global__ void cyclic_strip_fill_kernel(int64_t N, const int64_t *__restrict__ predptr,
                                         const uint16_t *__restrict__ pred, int64_t per,
                                         int64_t threads, uint32_t *__restrict__ strips) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (p >= N) return;
  for (int64_t e = predptr[p] + lane; e < predptr[p + 1]; e += 64) {
    const int64_t t = e / per, i = e - t * per;
    strips[i * threads + t] = ((uint32_t)p << 16) | (uint32_t)pred[e];
  }
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

constexpr int kChainThreads = 1024;

__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t *red) {
  for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, off));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint32_t r = red[0];
  for (int w = 1; w < kChainThreads / 64; ++w) r = min(r, red[w]);
  return r;
}

// The whole walk in one workgroup: x (16 bits) and the gathered minima (32
// bits, for LDS atomic min) live in LDS, the strips stream from L2.  Per
// level: every thread walks its strip, keeping the least x_q while the
// column stays the same and folding it into y[p] with one LDS atomic min when
// the column changes; after a barrier x_p = z_p + y_p (saturating) and the
// level's answer min_p x_p + end_p is reduced.  out[k - 1] for k = 1..nmax.
__global__ void __launch_bounds__(kChainThreads)
    cyclic_chain_kernel(int64_t N, int64_t nmax, int64_t per, const uint32_t *__restrict__ strips,
                        const uint8_t *__restrict__ z, const uint16_t *__restrict__ start,
                        const uint16_t *__restrict__ end, int32_t *__restrict__ out) {
  extern __shared__ uint32_t lds[];
  uint32_t *y = lds;                         // N
  uint16_t *x = (uint16_t *)(lds + N);       // N
  __shared__ uint32_t red[kChainThreads / 64];
  const int tid = threadIdx.x;
  uint32_t best = 0xFFFFu;
  for (int64_t p = tid; p < N; p += kChainThreads) {
    const uint16_t v = start[p];
    x[p] = v;
    y[p] = 0xFFFFu;
    best = min(best, min((uint32_t)v + (uint32_t)end[p], 0xFFFFu));
  }
  best = block_min_u32(best, red);
  if (tid == 0) out[0] = (int32_t)best;
  for (int64_t k = 2; k <= nmax; ++k) {
    __syncthreads();
    // the strip's entries eight at a time: the loads first, then the LDS
    // reads, then the column breaks (padding, 0xFFFFFFFF, only ends a strip
    // and reads x[0xFFFF & ...] of no column: its column 0xFFFF never matches)
    uint32_t cur_p = 0xFFFFFFFFu, cur = 0xFFFFu;
    for (int64_t i0 = 0; i0 < per; i0 += 8) {
      uint32_t e[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        e[j] = i0 + j < per ? strips[(i0 + j) * kChainThreads + tid] : 0xFFFFFFFFu;
      if (e[0] == 0xFFFFFFFFu) break;
      uint32_t v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = e[j] == 0xFFFFFFFFu ? 0xFFFFu : (uint32_t)x[e[j] & 0xFFFFu];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (e[j] == 0xFFFFFFFFu) break;
        const uint32_t p = e[j] >> 16;
        if (p != cur_p) {
          if (cur_p != 0xFFFFFFFFu) atomicMin(&y[cur_p], cur);
          cur_p = p;
          cur = v[j];
        } else {
          cur = min(cur, v[j]);
        }
      }
    }
    if (cur_p != 0xFFFFFFFFu) atomicMin(&y[cur_p], cur);
    __syncthreads();
    best = 0xFFFFu;
    for (int64_t p = tid; p < N; p += kChainThreads) {
      const uint32_t v = min(y[p] + (uint32_t)z[p], 0xFFFFu);
      x[p] = (uint16_t)v;
      y[p] = 0xFFFFu;
      best = min(best, min(v + (uint32_t)end[p], 0xFFFFu));
    }
    best = block_min_u32(best, red);
    if (tid == 0) out[k - 1] = (int32_t)best;
  }
}

// One level of the walk as two full-chip launches.  The predecessor lists
// are cut into items of at most kItemLen entries (the all-zero word alone has
// every word as a predecessor), one wave per item, longest lists first; a
// wave gathers its item's x_q with all its loads in flight and folds the
// least into ym[p] (32 bits, INF between levels) with one atomic.  Then
// y_p = z_p + ym[p] (saturating), ym[p] goes back to INF, and the level's
// answer min_p y_p + end_p folds into *out with one atomic per wave.
struct WalkItem {
  int64_t begin;
  int32_t p, len;
};

constexpr int kItemLen = 256;

__global__ void __launch_bounds__(256)
    cyclic_items_kernel(int64_t nitems, const WalkItem *__restrict__ items,
                        const uint16_t *__restrict__ pred, const uint16_t *__restrict__ x,
                        uint32_t *__restrict__ ym) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (w >= nitems) return;
  const WalkItem it = items[w];
  uint16_t q[kItemLen / 64];
#pragma unroll
  for (int j = 0; j < kItemLen / 64; ++j) {
    const int i = lane + 64 * j;
    q[j] = i < it.len ? pred[it.begin + i] : (uint16_t)0xFFFFu;
  }
  uint32_t best = 0xFFFFu;
#pragma unroll
  for (int j = 0; j < kItemLen / 64; ++j)
    if (q[j] != 0xFFFFu) best = min(best, (uint32_t)x[q[j]]);
  for (int off = 32; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off));
  if (lane == 0 && best < 0xFFFFu) atomicMin(&ym[it.p], best);
}

__global__ void __launch_bounds__(256)
    cyclic_finish_kernel(int64_t N, const uint8_t *__restrict__ z,
                         const uint16_t *__restrict__ end, uint32_t *__restrict__ ym,
                         uint16_t *__restrict__ y, int32_t *__restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t best = 0xFFFFu;
  if (p < N) {
    const uint32_t v = min(ym[p] + (uint32_t)z[p], 0xFFFFu);
    ym[p] = 0xFFFFu;
    y[p] = (uint16_t)v;
    best = min(v + (uint32_t)end[p], 0xFFFFu);
  }
  for (int off = 32; off > 0; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off));
  if ((threadIdx.x & 63) == 0 && best < 0xFFFFu) atomicMin(out, (int32_t)best);
}

// min_p x_p + end_p into *out (one workgroup; u16 vectors).
__global__ void __launch_bounds__(kChainThreads)
    cyclic_answer_kernel(int64_t N, const uint16_t *__restrict__ x,
                         const uint16_t *__restrict__ end, int32_t *__restrict__ out) {
  __shared__ uint32_t red[kChainThreads / 64];
  uint32_t best = 0xFFFFu;
  for (int64_t p = threadIdx.x; p < N; p += kChainThreads)
    best = min(best, min((uint32_t)x[p] + (uint32_t)end[p], 0xFFFFu));
  best = block_min_u32(best, red);
  if (threadIdx.x == 0) *out = (int32_t)best;
}

}  // namespace

int64_t cyclic_count_host(int m) {
  if (m < 3 || m > kMaxM) return -1;
  int32_t g[kMaxM - 1][9][9];
  build_cyclic_completions(m, g);
  int64_t s = 0;
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) s += g[m - 2][c * 3 + d][c * 3 + d];
  return s;
}

hipError_t launch_cyclic_words(int m, uint32_t *codes, uint8_t *zeros, uint32_t *masks,
                               hipStream_t s) {
  uint32_t total = 1;
  for (int i = 0; i < m; ++i) total *= 3u;
  const int bs = 256;
  hipLaunchKernelGGL(cyclic_words_kernel, dim3((total + bs - 1) / bs), dim3(bs), 0, s, m, total,
                     codes, zeros, masks);
  return hipGetLastError();
}

hipError_t launch_cyclic_dense(int m, int64_t N, const uint32_t *masks, int dtype, void *A,
                               int64_t lda, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const int bs = 256;
  dim3 grid((unsigned)N, (unsigned)std::min<int64_t>((N + bs - 1) / bs, 16));
  if (dtype == TP_U16)
    hipLaunchKernelGGL((cyclic_dense_kernel<uint16_t, kInf16>), grid, dim3(bs), 0, s, m, N, masks,
                       (uint16_t *)A, lda);
  else
    hipLaunchKernelGGL((cyclic_dense_kernel<uint8_t, kInf8>), grid, dim3(bs), 0, s, m, N, masks,
                       (uint8_t *)A, lda);
  return hipGetLastError();
}

hipError_t launch_cyclic_boundary(int m, int64_t N, const uint32_t *masks, int dtype, void *start,
                                  void *end, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const int bs = 256;
  dim3 grid((unsigned)((N + bs - 1) / bs));
  if (dtype == TP_U16)
    hipLaunchKernelGGL((cyclic_boundary_kernel<uint16_t, kInf16>), grid, dim3(bs), 0, s, m, N,
                       masks, (uint16_t *)start, (uint16_t *)end);
  else
    hipLaunchKernelGGL((cyclic_boundary_kernel<uint8_t, kInf8>), grid, dim3(bs), 0, s, m, N, masks,
                       (uint8_t *)start, (uint8_t *)end);
  return hipGetLastError();
}

hipError_t launch_cyclic_pred_count(int m, int64_t N, const uint32_t *masks, int64_t *predptr,
                                    hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(cyclic_pred_count_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, m,
                     N, masks, predptr);
  return hipGetLastError();
}

hipError_t launch_cyclic_pred_fill(int m, int64_t N, const uint32_t *masks, const int64_t *predptr,
                                   uint16_t *pred, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(cyclic_pred_fill_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, m, N,
                     masks, predptr, pred);
  return hipGetLastError();
}

int64_t cyclic_strip_length(int64_t nnz) {
  return std::max<int64_t>(1, (nnz + kChainThreads - 1) / kChainThreads);
}

size_t cyclic_chain_lds_bytes(int64_t N) { return (size_t)N * 6; }

hipError_t launch_cyclic_strips(int64_t N, int64_t nnz, const int64_t *predptr,
                                const uint16_t *pred, uint32_t *strips, hipStream_t s) {
  const int64_t per = cyclic_strip_length(nnz);
  const int64_t total = per * kChainThreads;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     strips, total, 0xFFFFFFFFu);
  if (N == 0) return hipGetLastError();
  hipLaunchKernelGGL(cyclic_strip_fill_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, N,
                     predptr, pred, per, (int64_t)kChainThreads, strips);
  return hipGetLastError();
}

hipError_t launch_cyclic_chain(int64_t N, int64_t nnz, int64_t nmax, const uint32_t *strips,
                               const uint8_t *z, const uint16_t *start, const uint16_t *end,
                               int32_t *out, hipStream_t s) {
  const size_t lds = cyclic_chain_lds_bytes(N);
  hipLaunchKernelGGL(cyclic_chain_kernel, dim3(1), dim3(kChainThreads), lds, s, N, nmax,
                     cyclic_strip_length(nnz), strips, z, start, end, out);
  return hipGetLastError();
}

int64_t cyclic_items_host(int64_t N, const int64_t *predptr, const int32_t *order,
                          std::vector<char> *bytes) {
  std::vector<WalkItem> items;
  for (int64_t w = 0; w < N; ++w) {
    const int32_t p = order[w];
    for (int64_t b = predptr[p]; b < predptr[p + 1]; b += kItemLen)
      items.push_back(WalkItem{b, p, (int32_t)std::min<int64_t>(kItemLen, predptr[p + 1] - b)});
  }
  bytes->assign((const char *)items.data(), (const char *)(items.data() + items.size()));
  return (int64_t)items.size();
}

hipError_t launch_cyclic_step(int64_t N, int64_t nitems, const void *items, const uint16_t *pred,
                              const uint8_t *z, const uint16_t *end, uint32_t *ym,
                              const uint16_t *x, uint16_t *y, int32_t *out, hipStream_t s) {
  if (N == 0) return hipSuccess;
  if (nitems > 0)
    hipLaunchKernelGGL(cyclic_items_kernel, dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s,
                       nitems, (const WalkItem *)items, pred, x, ym);
  hipLaunchKernelGGL(cyclic_finish_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N,
                     z, end, ym, y, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                     count, v);
  return hipGetLastError();
}

hipError_t launch_cyclic_answer(int64_t N, const uint16_t *x, const uint16_t *end, int32_t *out,
                                hipStream_t s) {
  hipLaunchKernelGGL(cyclic_answer_kernel, dim3(1), dim3(kChainThreads), 0, s, N, x, end, out);
  return hipGetLastError();
}

}  // namespace tp
