// Correct words, the "can follow" relation and the state matrix A(D_n)
// (Section 2.2 and Algorithm 1 of Section 3), built on the device.
//
// Words.  A word is correct when no inner position i (with both neighbours)
// holds 0 2 0 around it or a 1 between two non-zero letters (the patterns
// 020, 111, 211, 112, 212), it does not start with 1 followed by a non-zero
// letter (11, 12) and does not end with a non-zero letter followed by 1
// (11, 21).  These rules only look at windows of three letters, so the
// correct words form a regular language: the number of correct completions of
// a prefix depends only on its last two letters and on how many letters are
// left.  One thread per base-3 code x < 3^n tests x and, when it is correct,
// computes its rank among the correct words from that completion table, so
// the words land in increasing order without a prefix sum.
//
// Arcs.  Each word is kept as two n-bit masks, Z (letters equal to 0) and O
// (letters equal to 1); the 2s are the rest.  p can follow q when
//   every 2 of q sits over a 0 of p,
//   every 2 of p sees exactly one 0 among q_i, p_{i-1}, p_{i+1},
//   every 1 of p sees at least two 0s among them,
// with neighbours outside the path absent.  With x = Z(q), y = Z(p) << 1 and
// w = Z(p) >> 1 (both cut to n bits) the "exactly one" and "at least two"
// sets are bitwise functions of x, y, w, so the test is a handful of integer
// operations for all n positions at once.  The arc label is the number of
// zeros of p.
#include "device_core.hpp"

namespace tp {

namespace {

constexpr int kMaxN = 13;

__host__ __device__ inline bool window_ok(int a, int b, int c) {
  if (a == 0 && b == 2 && c == 0) return false;  // 020
  if (b == 1 && a != 0 && c != 0) return false;  // 111 211 112 212
  return true;
}
__host__ __device__ inline bool start_ok(int a, int b) { return !(a == 1 && b != 0); }
__host__ __device__ inline bool end_ok(int a, int b) { return !(b == 1 && a != 0); }

// f[r][a][b]: number of ways to append r letters after a prefix ending in
// letters a, b such that every new window and the end rule hold.
__host__ __device__ inline void build_completions(int n, int32_t (*f)[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) f[0][a][b] = end_ok(a, b) ? 1 : 0;
  for (int r = 1; r <= n - 2; ++r)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        int32_t s = 0;
        for (int c = 0; c < 3; ++c)
          if (window_ok(a, b, c)) s += f[r - 1][b][c];
        f[r][a][b] = s;
      }
}

__global__ void words_kernel(int n, uint32_t total, uint32_t *__restrict__ codes,
                             uint8_t *__restrict__ zeros, uint32_t *__restrict__ masks) {
  __shared__ int32_t f[kMaxN][3][3];
  if (threadIdx.x == 0 && n >= 2) build_completions(n, f);
  __syncthreads();
  uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total) return;
  int w[kMaxN];
  uint32_t t = x;
  for (int i = n - 1; i >= 0; --i) {
    w[i] = (int)(t % 3u);
    t /= 3u;
  }
  if (n >= 2) {
    if (!start_ok(w[0], w[1]) || !end_ok(w[n - 2], w[n - 1])) return;
    for (int i = 1; i + 1 < n; ++i)
      if (!window_ok(w[i - 1], w[i], w[i + 1])) return;
  }
  // rank = number of correct words that are smaller than x
  int64_t rank = 0;
  if (n == 1) {
    rank = w[0];
  } else {
    for (int c = 0; c < w[0]; ++c)
      for (int d = 0; d < 3; ++d)
        if (start_ok(c, d)) rank += f[n - 2][c][d];
    for (int i = 1; i < n; ++i) {
      for (int c = 0; c < w[i]; ++c) {
        bool ok = (i == 1) ? start_ok(w[0], c) : window_ok(w[i - 2], w[i - 1], c);
        if (ok) rank += f[n - 1 - i][w[i - 1]][c];
      }
    }
  }
  uint32_t zm = 0, om = 0;
  for (int i = 0; i < n; ++i) {
    zm |= (w[i] == 0 ? 1u : 0u) << i;
    om |= (w[i] == 1 ? 1u : 0u) << i;
  }
  if (codes) codes[rank] = x;
  if (zeros) zeros[rank] = (uint8_t)__builtin_popcount(zm);
  if (masks) masks[rank] = zm | (om << 16);
}

template <typename T, T INF>
__global__ void dense_state_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                   T *__restrict__ A, int64_t lda) {
  // block (q, y) fills columns [4 * y * blockDim.x, 4 * (y + 1) * blockDim.x) of row q
  const int64_t q = blockIdx.x;
  const uint32_t mq = masks[q];
  T *row = A + q * lda;
  const int64_t p_begin = (int64_t)blockIdx.y * blockDim.x * 4;
  for (int t = 0; t < 4; ++t) {
    const int64_t p = p_begin + (int64_t)t * blockDim.x + threadIdx.x;
    if (p >= N) break;
    const uint32_t mp = masks[p];
    row[p] = can_follow(mq, mp, full) ? (T)__builtin_popcount(mp & 0xFFFFu) : INF;
  }
}

// One wave per row: out-degree of q.
__global__ void csr_count_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                 int64_t *__restrict__ rowptr) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (q >= N) return;
  const uint32_t mq = masks[q];
  int64_t cnt = 0;
  for (int64_t p0 = 0; p0 < N; p0 += 64) {
    int64_t p = p0 + lane;
    bool arc = (p < N) && can_follow(mq, masks[p], full);
    cnt += __popcll(__ballot(arc));
  }
  if (lane == 0) {
    rowptr[q + 1] = cnt;
    if (q == 0) rowptr[0] = 0;
  }
}

// One workgroup: in-place inclusive scan of rowptr[1..N] (counts -> offsets).
__global__ void __launch_bounds__(1024) scan_kernel(int64_t N, int64_t *__restrict__ rowptr) {
  __shared__ int64_t part[1024];
  __shared__ int64_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  constexpr int PER = 4;
  const int64_t chunk = 1024 * PER;
  for (int64_t base = 1; base <= N; base += chunk) {
    int64_t v[PER];
    int64_t local = 0;
    for (int t = 0; t < PER; ++t) {
      int64_t idx = base + (int64_t)threadIdx.x * PER + t;
      v[t] = (idx <= N) ? rowptr[idx] : 0;
      local += v[t];
    }
    part[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int64_t add = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += add;
      __syncthreads();
    }
    int64_t run = carry_s + part[threadIdx.x] - local;
    for (int t = 0; t < PER; ++t) {
      int64_t idx = base + (int64_t)threadIdx.x * PER + t;
      run += v[t];
      if (idx <= N) rowptr[idx] = run;
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry_s += part[1023];
    __syncthreads();
  }
}

// One wave per row: successor indices in increasing order; colz, when not
// NULL, gets each successor p with its label z_p (zeros of word p) in the
// top byte (N < 2^24 for every n <= 12).
__global__ void csr_fill_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                const int64_t *__restrict__ rowptr, uint32_t *__restrict__ col,
                                uint32_t *__restrict__ colz) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (q >= N) return;
  const uint32_t mq = masks[q];
  int64_t pos = rowptr[q];
  for (int64_t p0 = 0; p0 < N; p0 += 64) {
    int64_t p = p0 + lane;
    bool arc = (p < N) && can_follow(mq, masks[p], full);
    uint64_t b = __ballot(arc);
    if (arc) {
      uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      col[pos + below] = (uint32_t)p;
      if (colz)
        colz[pos + below] = (uint32_t)p | ((uint32_t)__builtin_popcount(masks[p] & 0xFFFFu) << 24);
    }
    pos += __popcll(b);
  }
}

}  // namespace

int64_t word_count_host(int n) {
  if (n < 1 || n > kMaxN) return -1;
  if (n == 1) return 3;
  int32_t f[kMaxN][3][3];
  build_completions(n, f);
  int64_t s = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (start_ok(a, b)) s += f[n - 2][a][b];
  return s;
}

hipError_t launch_words(int n, uint32_t *codes, uint8_t *zeros, uint32_t *masks, hipStream_t s) {
  uint32_t total = 1;
  for (int i = 0; i < n; ++i) total *= 3u;
  const int bs = 256;
  hipLaunchKernelGGL(words_kernel, dim3((total + bs - 1) / bs), dim3(bs), 0, s, n, total, codes,
                     zeros, masks);
  return hipGetLastError();
}

hipError_t launch_dense_state(int n, int64_t N, const uint32_t *masks, int dtype, void *A,
                              int64_t lda, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int bs = 256;
  dim3 grid((unsigned)N, (unsigned)((N + bs * 4 - 1) / (bs * 4)));
  if (dtype == TP_U16)
    hipLaunchKernelGGL((dense_state_kernel<uint16_t, kInf16>), grid, dim3(bs), 0, s, N, full,
                       masks, (uint16_t *)A, lda);
  else
    hipLaunchKernelGGL((dense_state_kernel<uint8_t, kInf8>), grid, dim3(bs), 0, s, N, full, masks,
                       (uint8_t *)A, lda);
  return hipGetLastError();
}

hipError_t launch_csr_count(int64_t N, int n, const uint32_t *masks, int64_t *rowptr,
                            hipStream_t s) {
  if (N == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int waves = 4;
  hipLaunchKernelGGL(csr_count_kernel, dim3((unsigned)((N + waves - 1) / waves)), dim3(64 * waves),
                     0, s, N, full, masks, rowptr);
  return hipGetLastError();
}

hipError_t launch_scan_rowptr(int64_t N, int64_t *rowptr, hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, N, rowptr);
  return hipGetLastError();
}

hipError_t launch_csr_fill(int64_t N, int n, const uint32_t *masks, const int64_t *rowptr,
                           uint32_t *col, uint32_t *colz, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int waves = 4;
  hipLaunchKernelGGL(csr_fill_kernel, dim3((unsigned)((N + waves - 1) / waves)), dim3(64 * waves),
                     0, s, N, full, masks, rowptr, col, colz);
  return hipGetLastError();
}

}  // namespace tp
