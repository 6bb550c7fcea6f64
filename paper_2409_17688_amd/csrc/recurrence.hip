// Recurrence of the powers of A = A(D_n) (Lemma 1, Theorem 3) and the
// searches of Algorithms 3 and 4, with Algorithm 5's diagonal minima.
//
// Lemma 1: once A^(n0 + a) = b (x) A^n0 (every entry of the later power is
// the earlier one plus the constant b, INF entries matching), the same holds
// for every later pair at distance a; Theorem 3 turns it into the finite
// difference equation gamma_2(m + a) = gamma_2(m) + b for m >= n0.
//
// Device side: one chain A^k = A x A^(k-1) (the library's sparse left step)
// through a ring of window + 1 powers; after each step the new power is
// compared with the `window` powers before it by a constant-difference
// reduction, and its diagonal minimum is taken.  The comparison is a pure
// stream over 2 N^2 entries per pair (HBM bound): one wave per row, lanes on
// 16-byte chunks, the new power's chunk loaded once for up to kMaxCmp earlier
// powers, {min, max} of the finite differences per pair, INF patterns that
// disagree forcing min < max.  Partial results per workgroup go to a small
// buffer and a one-block kernel folds them, so there are no atomics.
// Host side: Algorithms 3 and 4 on the table of comparison results.
#include <limits.h>

#include <algorithm>
#include <vector>

#include "device_core.hpp"

namespace tp {

namespace {

constexpr int kMaxCmp = 8;           // earlier powers compared in one pass
constexpr int kCmpBlocks = 2048;     // workgroups of one pass (4 rows each at a time)
constexpr int32_t kMismatch = 1 << 30;
constexpr int kMaxWindow = 256;      // earlier powers each power is compared with, at most

struct CmpSet {
  const uint16_t *y[kMaxCmp];
};

__device__ __forceinline__ void fold_pair(uint32_t x2, uint32_t y2, int valid, int32_t &mn,
                                          int32_t &mx) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int32_t x = (int32_t)((x2 >> (16 * h)) & 0xFFFFu);
    const int32_t y = (int32_t)((y2 >> (16 * h)) & 0xFFFFu);
    const bool xi = x == 0xFFFF, yi = y == 0xFFFF;
    int32_t lo = INT_MAX, hi = INT_MIN;
    if (h < valid) {
      if (xi != yi) {
        lo = -kMismatch;
        hi = kMismatch;
      } else if (!xi) {
        lo = hi = x - y;
      }
    }
    mn = min(mn, lo);
    mx = max(mx, hi);
  }
}

// partial[block][2 d], partial[block][2 d + 1] = {min, max} of X - Y_d over
// the rows this workgroup visited
__global__ void __launch_bounds__(256) const_diff_kernel(int64_t N, const uint16_t *X, int64_t ld,
                                                         CmpSet set, int nd, int32_t *partial) {
  __shared__ int32_t red[4][2 * kMaxCmp];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int32_t mn[kMaxCmp], mx[kMaxCmp];
#pragma unroll
  for (int d = 0; d < kMaxCmp; ++d) {
    mn[d] = INT_MAX;
    mx[d] = INT_MIN;
  }
  const gconst<u32x4> Xg = (gconst<u32x4>)to_global(X);
  const int64_t ld8 = ld / 8, chunks = (N + 7) / 8;
  // kUnroll chunks per lane per round, their loads issued before any is used
  constexpr int kUnroll = 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < N; r += (int64_t)gridDim.x * 4) {
    for (int64_t c0 = lane; c0 < chunks; c0 += 64 * kUnroll) {
      u32x4 xv[kUnroll];
      int valid[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t c = c0 + 64 * u;
        valid[u] = c >= chunks ? 0 : (N - c * 8 < 8 ? (int)(N - c * 8) : 8);
        xv[u] = c < chunks ? Xg[r * ld8 + c] : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int d = 0; d < kMaxCmp; ++d) {
        if (d < nd) {
          const gconst<u32x4> Yg = (gconst<u32x4>)to_global(set.y[d]);
          u32x4 yv[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int64_t c = c0 + 64 * u;
            yv[u] = c < chunks ? Yg[r * ld8 + c] : u32x4{0u, 0u, 0u, 0u};
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            fold_pair(xv[u].x, yv[u].x, valid[u], mn[d], mx[d]);
            fold_pair(xv[u].y, yv[u].y, valid[u] - 2, mn[d], mx[d]);
            fold_pair(xv[u].z, yv[u].z, valid[u] - 4, mn[d], mx[d]);
            fold_pair(xv[u].w, yv[u].w, valid[u] - 6, mn[d], mx[d]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < kMaxCmp; ++d) {
    for (int o = 32; o >= 1; o >>= 1) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], o, 64));
      mx[d] = max(mx[d], __shfl_xor(mx[d], o, 64));
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < kMaxCmp; ++d) {
      red[wave][2 * d] = mn[d];
      red[wave][2 * d + 1] = mx[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMaxCmp) {
    const int v = threadIdx.x;
    int32_t acc = red[0][v];
    for (int w = 1; w < 4; ++w) acc = (v & 1) ? max(acc, red[w][v]) : min(acc, red[w][v]);
    partial[(int64_t)blockIdx.x * 2 * kMaxCmp + v] = acc;
  }
}

// out[2 d], out[2 d + 1] = fold of partial[*][2 d], partial[*][2 d + 1], d < nd
__global__ void __launch_bounds__(256) const_diff_fold_kernel(const int32_t *partial, int blocks,
                                                              int nd, int32_t *out) {
  __shared__ int32_t red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = 0; v < 2 * nd; ++v) {
    const bool is_max = v & 1;
    int32_t acc = is_max ? INT_MIN : INT_MAX;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) {
      const int32_t p = partial[(int64_t)b * 2 * kMaxCmp + v];
      acc = is_max ? max(acc, p) : min(acc, p);
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const int32_t t = __shfl_xor(acc, o, 64);
      acc = is_max ? max(acc, t) : min(acc, t);
    }
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t r = red[0];
      for (int w = 1; w < 4; ++w) r = is_max ? max(r, red[w]) : min(r, red[w]);
      out[v] = r;
    }
    __syncthreads();
  }
}

// The same reduction on shared-base compact powers (every entry finite):
// {min, max} of (G_x + x) - (G_y + y) = G_x - G_y + (x - y), lanes on 16-byte
// chunks of residuals.
struct CmpSet8 {
  const uint8_t *y[kMaxCmp];
  const int32_t *by[kMaxCmp];
};

__device__ __forceinline__ void fold_bytes(uint32_t x4, uint32_t y4, int valid, int32_t &mn,
                                           int32_t &mx) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    if (h < valid) {
      const int32_t d = (int32_t)((x4 >> (8 * h)) & 0xFFu) - (int32_t)((y4 >> (8 * h)) & 0xFFu);
      mn = min(mn, d);
      mx = max(mx, d);
    }
  }
}

__global__ void __launch_bounds__(256) const_diff8_kernel(int64_t N, const uint8_t *X,
                                                          const int32_t *bx, int64_t ld,
                                                          CmpSet8 set, int nd, int32_t *partial) {
  __shared__ int32_t red[4][2 * kMaxCmp];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  int32_t mn[kMaxCmp], mx[kMaxCmp];
#pragma unroll
  for (int d = 0; d < kMaxCmp; ++d) {
    mn[d] = INT_MAX;
    mx[d] = INT_MIN;
  }
  const gconst<u32x4> Xg = (gconst<u32x4>)to_global(X);
  const int64_t ld16 = ld / 16, chunks = (N + 15) / 16;
  constexpr int kUnroll = 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < N; r += (int64_t)gridDim.x * 4) {
    for (int64_t c0 = lane; c0 < chunks; c0 += 64 * kUnroll) {
      u32x4 xv[kUnroll];
      int valid[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t c = c0 + 64 * u;
        valid[u] = c >= chunks ? 0 : (N - c * 16 < 16 ? (int)(N - c * 16) : 16);
        xv[u] = c < chunks ? Xg[r * ld16 + c] : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int d = 0; d < kMaxCmp; ++d) {
        if (d < nd) {
          const gconst<u32x4> Yg = (gconst<u32x4>)to_global(set.y[d]);
          u32x4 yv[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int64_t c = c0 + 64 * u;
            yv[u] = c < chunks ? Yg[r * ld16 + c] : u32x4{0u, 0u, 0u, 0u};
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            fold_bytes(xv[u].x, yv[u].x, valid[u], mn[d], mx[d]);
            fold_bytes(xv[u].y, yv[u].y, valid[u] - 4, mn[d], mx[d]);
            fold_bytes(xv[u].z, yv[u].z, valid[u] - 8, mn[d], mx[d]);
            fold_bytes(xv[u].w, yv[u].w, valid[u] - 12, mn[d], mx[d]);
          }
        }
      }
    }
  }
  const int32_t gx = ((kconst_i32)bx)[0];
#pragma unroll
  for (int d = 0; d < kMaxCmp; ++d) {
    for (int o = 32; o >= 1; o >>= 1) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], o, 64));
      mx[d] = max(mx[d], __shfl_xor(mx[d], o, 64));
    }
    if (d < nd && mn[d] != INT_MAX) {
      const int32_t shift = gx - ((kconst_i32)set.by[d])[0];
      mn[d] += shift;
      mx[d] += shift;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < kMaxCmp; ++d) {
      red[wave][2 * d] = mn[d];
      red[wave][2 * d + 1] = mx[d];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMaxCmp) {
    const int v = threadIdx.x;
    int32_t acc = red[0][v];
    for (int w = 1; w < 4; ++w) acc = (v & 1) ? max(acc, red[w][v]) : min(acc, red[w][v]);
    partial[(int64_t)blockIdx.x * 2 * kMaxCmp + v] = acc;
  }
}

int cmp_blocks(int64_t N) { return (int)std::max<int64_t>(1, std::min<int64_t>((N + 3) / 4, kCmpBlocks)); }

// {min, max} of X - Y_d for the nd <= kMaxCmp powers in `set` into out[0 .. 2 nd)
hipError_t launch_const_diff(int64_t N, const uint16_t *X, int64_t ld, const CmpSet &set, int nd,
                             int32_t *partial, int32_t *out, hipStream_t s) {
  const int blocks = cmp_blocks(N);
  hipLaunchKernelGGL(const_diff_kernel, dim3(blocks), dim3(256), 0, s, N, X, ld, set, nd, partial);
  hipLaunchKernelGGL(const_diff_fold_kernel, dim3(1), dim3(256), 0, s, (const int32_t *)partial,
                     blocks, nd, out);
  return hipGetLastError();
}

hipError_t launch_const_diff8(int64_t N, const uint8_t *X, const int32_t *bx, int64_t ld,
                              const CmpSet8 &set, int nd, int32_t *partial, int32_t *out,
                              hipStream_t s) {
  const int blocks = cmp_blocks(N);
  hipLaunchKernelGGL(const_diff8_kernel, dim3(blocks), dim3(256), 0, s, N, X, bx, ld, set, nd,
                     partial);
  hipLaunchKernelGGL(const_diff_fold_kernel, dim3(1), dim3(256), 0, s, (const int32_t *)partial,
                     blocks, nd, out);
  return hipGetLastError();
}

// Algorithm 3's test on a folded {min, max}: holds with b = min when the
// difference is constant, with b = 0 when no entry is finite
bool const_holds(const int32_t *mm, int64_t *b) {
  if (mm[0] == INT_MAX && mm[1] == INT_MIN) {
    *b = 0;
    return true;
  }
  if (mm[0] != mm[1]) return false;
  *b = mm[0];
  return true;
}

struct DevMem {
  void *p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
};

// Algorithms 3 and 4 on the comparison table: table[(i W + d - 1) 2 ..] is
// the folded {min, max} of A^i - A^(i-d), 1 <= d <= min(W, i - 1).
tp_recurrence_t search(const std::vector<int32_t> &table, int K, int W) {
  auto holds = [&](int i, int d, int64_t *b) {
    return const_holds(&table[((size_t)i * W + (d - 1)) * 2], b);
  };
  tp_recurrence_t r{};
  r.K = K;
  r.window = W;
  // Algorithm 3: i from K down, j = i - d from i - 1 down (d up); a window
  // shorter than i - 1 leaves pairs of this i unexamined, so the search can
  // only continue past i when it covers them all
  for (int i = K; i >= 2 && !r.found; --i) {
    for (int d = 1; d <= std::min(W, i - 1); ++d) {
      int64_t b = 0;
      if (holds(i, d, &b)) {
        r.found = 1;
        r.a = d;
        r.b = b;
        r.r0 = i - d;
        break;
      }
    }
    if (!r.found && W < i - 1) {
      r.window_short = 1;
      break;
    }
  }
  // Algorithm 4: down from i = r0 + a while A^i = b (x) A^(i-a)
  r.n0 = -1;
  if (r.found) {
    for (int64_t i = r.r0 + r.a; i - r.a >= 1; --i) {
      int64_t b = 0;
      if (!holds((int)i, (int)r.a, &b) || b != r.b) break;
      r.n0 = i - r.a;
    }
  }
  return r;
}

constexpr int kNotHeld = 1;  // the compact chain cannot hold these powers
constexpr int kMaxEarly = 3;  // 16-bit powers before the switch, at most

int window_fit(int window, int K, size_t pbytes, size_t reserved, int *W) {
  *W = window > 0 ? std::min(window, K - 1) : std::min(K - 1, kMaxWindow);
  size_t free_b = 0, total_b = 0;
  TP_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
  const size_t margin = ((size_t)1 << 30) + reserved;
  const size_t avail = free_b > margin ? free_b - margin : 0;
  const size_t fit = pbytes ? avail / pbytes : (size_t)K;
  if (window == 0) {
    *W = (int)std::min<size_t>((size_t)*W, fit > 0 ? fit - 1 : 0);
    if (*W < 1) {
      set_error("two powers (%zu bytes each) do not fit", pbytes);
      return TP_ENOMEM;
    }
  } else if ((size_t)*W + 1 > fit) {
    set_error("window %d needs %zu bytes of powers; %zu free", *W, (*W + 1) * pbytes, avail);
    return TP_ENOMEM;
  }
  return TP_OK;
}

// The recurrence with the chain on shared-base compact powers.  A^1 .. A^k0
// run in 16 bits until a power converts (every entry finite, span <= 254);
// the earlier ones hold INF entries, so against any later (all finite) power
// their INF patterns disagree and the pair's entry is {-M, M}, as the 16-bit
// comparison makes it.  From k0 on the chain, diagonal minima and
// comparisons run on the compact ring.  kNotHeld when a power cannot be held
// (the caller then runs the 16-bit chain).
int recurrence_compact(const StateView &v, int K, int window, tp_recurrence_t *out,
                       int32_t *diag_min_host, hipStream_t stream) {
  const int n = v.n;
  const int64_t N = v.N, ld = (N + 63) / 64 * 64;
  const size_t p16 = (size_t)N * (size_t)ld * sizeof(uint16_t), p8 = (size_t)N * (size_t)ld;
  if (K <= kMaxEarly) return kNotHeld;
  int W = 0;
  // the window the 16-bit chain would take (the same comparisons, so the
  // same search and the same reported window); the compact ring then uses
  // half of that memory
  int rc = window_fit(window, K, p16, 0, &W);
  if (rc != TP_OK) return rc;
  std::vector<int32_t> table((size_t)(K + 1) * W * 2, 0), diag((size_t)K + 1, 0);

  DevMem res, dg, partial, st, early[kMaxEarly + 1], conv, cbase;
  TP_HIP_CHECK(hipMalloc(&res.p, (size_t)(K + 1) * W * 2 * sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&dg.p, (size_t)(K + 1) * sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&partial.p, (size_t)kCmpBlocks * 2 * kMaxCmp * sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&st.p, sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&cbase.p, 2 * sizeof(int32_t)));
  int32_t *resd = (int32_t *)res.p;

  // 16-bit powers until one converts
  int k0 = 0;
  for (int k = 1; k <= kMaxEarly && !k0; ++k) {
    TP_HIP_CHECK(hipMalloc(&early[k].p, p16));
    uint16_t *Y = (uint16_t *)early[k].p;
    if (k == 1)
      TP_HIP_CHECK(launch_dense_state(n, N, v.masks, TP_U16, Y, ld, stream));
    else
      TP_HIP_CHECK(state_step_view(v, (const uint16_t *)early[k - 1].p, ld, Y, ld, N, stream));
    TP_HIP_CHECK(launch_trace_min(TP_U16, N, Y, ld, (int32_t *)dg.p + k, stream));
    const int dmax = std::min(W, k - 1);
    if (dmax >= 1) {
      CmpSet set{};
      for (int j = 0; j < dmax; ++j) set.y[j] = (const uint16_t *)early[k - 1 - j].p;
      TP_HIP_CHECK(launch_const_diff(N, Y, ld, set, dmax, (int32_t *)partial.p,
                                     resd + (int64_t)k * W * 2, stream));
    }
    if (!conv.p) TP_HIP_CHECK(hipMalloc(&conv.p, p8));
    TP_HIP_CHECK(launch_fill_i32((int32_t *)st.p, 1, 0, stream));
    TP_HIP_CHECK(launch_shared_from_u16(N, N, Y, ld, (uint8_t *)conv.p, ld, (int32_t *)cbase.p,
                                        (int32_t *)st.p, stream));
    int32_t status = 0;
    TP_HIP_CHECK(hipMemcpyAsync(&status, st.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    TP_HIP_CHECK(hipStreamSynchronize(stream));
    if (status == 0) k0 = k;
    else if (!(status & 2)) return kNotHeld;  // finite but too wide: no INF argument
  }
  if (!k0) return kNotHeld;
  for (int k = 1; k <= k0; ++k) early[k].release();

  const int slots = W + 1;
  DevMem ring, bases;
  TP_HIP_CHECK(hipMalloc(&ring.p, p8 * slots));
  TP_HIP_CHECK(hipMalloc(&bases.p, (size_t)slots * 2 * sizeof(int32_t)));
  auto slot = [&](int k) { return (uint8_t *)ring.p + (size_t)(k % slots) * p8; };
  auto base = [&](int k) { return (int32_t *)bases.p + (size_t)(k % slots) * 2; };
  TP_HIP_CHECK(hipMemcpyAsync(slot(k0), conv.p, p8, hipMemcpyDeviceToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(base(k0), cbase.p, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              stream));
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  conv.release();
  TP_HIP_CHECK(launch_fill_i32((int32_t *)st.p, 1, 0, stream));

  for (int k = k0 + 1; k <= K; ++k) {
    TP_HIP_CHECK(launch_shared_step(v, slot(k - 1), ld, base(k - 1), slot(k), ld, base(k), N,
                                    (int32_t *)st.p, stream));
    TP_HIP_CHECK(launch_shared_diag(N, slot(k), ld, base(k), (int32_t *)dg.p + k, stream));
    const int dmax = std::min(W, k - k0);  // compact powers in the window
    for (int d0 = 1; d0 <= dmax; d0 += kMaxCmp) {
      const int nd = std::min(kMaxCmp, dmax - d0 + 1);
      CmpSet8 set{};
      for (int j = 0; j < nd; ++j) {
        set.y[j] = slot(k - (d0 + j));
        set.by[j] = base(k - (d0 + j));
      }
      TP_HIP_CHECK(launch_const_diff8(N, slot(k), base(k), ld, set, nd, (int32_t *)partial.p,
                                      resd + ((int64_t)k * W + (d0 - 1)) * 2, stream));
    }
  }
  int32_t status = 0;
  TP_HIP_CHECK(hipMemcpyAsync(table.data(), res.p, table.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipMemcpyAsync(diag.data(), dg.p, diag.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipMemcpyAsync(&status, st.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  if (status != 0) return kNotHeld;
  // pairs of a compact power with an early one: INF patterns disagree
  for (int k = k0 + 1; k <= K; ++k)
    for (int d = k - k0 + 1; d <= std::min(W, k - 1); ++d) {
      table[((size_t)k * W + (d - 1)) * 2] = -kMismatch;
      table[((size_t)k * W + (d - 1)) * 2 + 1] = kMismatch;
    }
  for (int k = 1; k <= K; ++k) diag_min_host[k - 1] = diag[k];
  *out = search(table, K, W);
  return TP_OK;
}

}  // namespace

}  // namespace tp

using namespace tp;

extern "C" {

int tp_const_diff(int64_t N, const void *d_X, int64_t ldx, const void *d_Y, int64_t ldy,
                  int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && N < (int64_t)1 << 31, "N = %lld out of range", (long long)N);
  TP_REQUIRE(d_out != nullptr, "d_out is NULL");
  TP_REQUIRE(N == 0 || (d_X != nullptr && d_Y != nullptr), "NULL matrix");
  TP_REQUIRE(ldx >= N && ldy >= N, "leading dimension below N");
  TP_REQUIRE(ldx == ldy && ldx % 8 == 0 && (uintptr_t)d_X % 16 == 0 && (uintptr_t)d_Y % 16 == 0,
             "X and Y need one leading dimension, a multiple of 8, and 16-byte alignment");
  DevMem partial;
  TP_HIP_CHECK(hipMallocAsync(&partial.p, (size_t)kCmpBlocks * 2 * kMaxCmp * sizeof(int32_t),
                              stream));
  CmpSet set{};
  set.y[0] = (const uint16_t *)d_Y;
  const hipError_t e = launch_const_diff(N, (const uint16_t *)d_X, ldx, set, 1,
                                         (int32_t *)partial.p, d_out, stream);
  const hipError_t f = hipFreeAsync(partial.p, stream);
  partial.p = nullptr;
  TP_HIP_CHECK(e);
  TP_HIP_CHECK(f);
  return TP_OK;
}

int tp_recurrence(int n, int K, int window, tp_recurrence_t *out, int32_t *diag_min_host,
                  hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(K >= 2 && K <= 65535, "K = %d outside 2..65535", K);
  TP_REQUIRE(window >= 0 && window <= kMaxWindow, "window = %d outside 0..%d", window,
             kMaxWindow);
  TP_REQUIRE(out != nullptr && diag_min_host != nullptr, "NULL output");
  if ((int64_t)n * K >= 0xFFFF) {
    set_error("n * K = %lld reaches the u16 INF", (long long)n * K);
    return TP_EOVERFLOW;
  }
  StateView v{};
  int rc = state_view(n, stream, &v);
  if (rc != TP_OK) return rc;
  if (compact_chain(n)) {
    rc = recurrence_compact(v, K, window, out, diag_min_host, stream);
    if (rc != kNotHeld) return rc;
  }
  const int64_t N = v.N, ld = (N + 63) / 64 * 64;
  const size_t pbytes = (size_t)N * (size_t)ld * sizeof(uint16_t);

  // window: explicit (clamped to K - 1) or the most of K - 1 that fits
  int W = 0;
  rc = window_fit(window, K, pbytes, 0, &W);
  if (rc != TP_OK) return rc;
  const int slots = W + 1;

  DevMem ring, res, dg, partial;
  TP_HIP_CHECK(hipMalloc(&ring.p, pbytes * slots));
  TP_HIP_CHECK(hipMalloc(&res.p, (size_t)(K + 1) * W * 2 * sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&dg.p, (size_t)(K + 1) * sizeof(int32_t)));
  TP_HIP_CHECK(hipMalloc(&partial.p, (size_t)kCmpBlocks * 2 * kMaxCmp * sizeof(int32_t)));
  auto slot = [&](int k) { return (uint16_t *)((char *)ring.p + (size_t)(k % slots) * pbytes); };
  int32_t *resd = (int32_t *)res.p;

  for (int k = 1; k <= K; ++k) {
    uint16_t *Y = slot(k);
    if (k == 1)
      TP_HIP_CHECK(launch_dense_state(n, N, v.masks, TP_U16, Y, ld, stream));
    else
      TP_HIP_CHECK(state_step_view(v, slot(k - 1), ld, Y, ld, N, stream));
    TP_HIP_CHECK(launch_trace_min(TP_U16, N, Y, ld, (int32_t *)dg.p + k, stream));
    const int dmax = std::min(W, k - 1);
    for (int d0 = 1; d0 <= dmax; d0 += kMaxCmp) {
      const int nd = std::min(kMaxCmp, dmax - d0 + 1);
      CmpSet set{};
      for (int j = 0; j < nd; ++j) set.y[j] = slot(k - (d0 + j));
      TP_HIP_CHECK(launch_const_diff(N, Y, ld, set, nd, (int32_t *)partial.p,
                                     resd + ((int64_t)k * W + (d0 - 1)) * 2, stream));
    }
  }
  std::vector<int32_t> table((size_t)(K + 1) * W * 2, 0), diag((size_t)K + 1, 0);
  TP_HIP_CHECK(hipMemcpyAsync(table.data(), res.p, table.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipMemcpyAsync(diag.data(), dg.p, diag.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, stream));
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  for (int k = 1; k <= K; ++k) diag_min_host[k - 1] = diag[k];
  *out = search(table, K, W);
  return TP_OK;
}

int tp_gamma2_recurrence(const tp_recurrence_t *rec, const int32_t *diag_min, int64_t m,
                         int64_t *gamma2) {
  TP_REQUIRE(rec != nullptr && diag_min != nullptr && gamma2 != nullptr, "NULL argument");
  TP_REQUIRE(m >= 3, "the cycle order m = %lld is below 3", (long long)m);
  if (m <= rec->K) {
    *gamma2 = diag_min[m - 1];
    return TP_OK;
  }
  TP_REQUIRE(rec->found && rec->a >= 1 && rec->n0 >= 1 && rec->n0 + rec->a - 1 <= rec->K,
             "m = %lld is beyond the %d powers and no recurrence is known", (long long)m,
             rec->K);
  const int64_t q = (m - rec->n0) / rec->a, r = (m - rec->n0) % rec->a;
  *gamma2 = (int64_t)diag_min[rec->n0 + r - 1] + q * rec->b;
  return TP_OK;
}

}  // extern "C"
