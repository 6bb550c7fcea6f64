// Compact powers: the chain step on 8-bit residuals with one offset per row.
//
// A power P of A(D_n) is held as
//   P[q][c] = R[q] + x[q][c],   x in 0..254 (u8),   R[q] int32,
// half the bytes of the 16-bit form, with a row whose entries are all INF
// held as R[q] = kDead and x = 255.  A row can be held when its entries are
// all finite and span at most 254; a row with both finite and INF entries,
// or a wider one, is reported by the conversion.  The powers of A(D_n) reach
// that shape after a few steps (every state then reaches every other, and
// the entries of a row differ by a few units).
//
// The left step Y = A(D_n) x X keeps the form.  Row q's offset is
//   R_Y[q] = min over successors p of q of (z_p + R_X[p]),
// a (min,+) product of A with the offsets (Section 2.2: the arc label z_p
// depends on the successor only), and the residuals are
//   y[q][c] = min over p of (z_p + R_X[p] - R_Y[q] + x[p][c]).
// With p* the successor that gives R_Y[q], y[q][c] <= x[p*][c]: residuals
// never grow from one power to the next and rows stay finite, so a held
// power's successors can be held too.  The shifts z_p + R_X[p] - base are
// per-entry constants, so the step is the blocked gather of blockstep.hip
// (16 rows per block, the union of their successor lists, one add per entry
// shared by the block's rows, then mins) on half the gathered bytes; base is
// the least offset of the block's rows and each row subtracts its own offset
// at the store.  Offsets are exact integers: P[q][c] above 65535 is INF only
// when expanded to the 16-bit form, as the 16-bit chain saturates there.
#include <algorithm>
#include <atomic>

#include "device_core.hpp"

namespace tp {

namespace {

constexpr int kRows = 16;                // rows per block (the blocked form's)
constexpr int32_t kDead = 0x3FFFFFFF;    // offset of an all-INF row
constexpr int32_t kMaxGap = 0xFF00;      // largest offset gap inside a block
constexpr int32_t kStatusRange = 1;      // a residual above 254 or a gap above kMaxGap
constexpr int32_t kStatusMixed = 2;      // a row with finite and INF entries

std::atomic<int> g_unroll{8};   // entries per round of the step (4 or 8)
std::atomic<int> g_grouped{1};  // shared-base step: block entries a mask group at a time

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// R_Y[q] = min over successors p (CSR with labels in the top byte) of
// z_p + R_X[p], over live successors only; kDead when none is live.  One
// wave per row.
__global__ void __launch_bounds__(256) compact_offsets_kernel(int64_t N, const int64_t *rowptr,
                                                              const uint32_t *colz,
                                                              const int32_t *RX, int32_t *RY) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= N) return;
  const gconst<int32_t> rx = to_global(RX);
  const gconst<uint32_t> cz = to_global(colz);
  int32_t m = kDead;
  for (int64_t e = rowptr[q] + lane; e < rowptr[q + 1]; e += 64) {
    const uint32_t c = cz[e];
    const int32_t r = rx[c & 0xFFFFFFu];
    if (r < kDead) m = min(m, r + (int32_t)(c >> 24));
  }
  m = wave_min_i32(m);
  if (lane == 0) RY[q] = m;
}

// Four residuals (bytes of w) as two packed 16-bit pairs.
__device__ __forceinline__ void unpack8(uint32_t w, u16x2 &lo, u16x2 &hi) {
  lo = as_pk(__builtin_amdgcn_perm(0u, w, 0x0c010c00u));
  hi = as_pk(__builtin_amdgcn_perm(0u, w, 0x0c030c02u));
}

// acc[r] = min(acc[r], lab + v) for the rows r whose bit is set in m.
__device__ __forceinline__ void apply_entry(u16x2 (&acc)[kRows][4], uint32_t m, u16x2 lab,
                                            const u16x2 (&v)[4]) {
  u16x2 s[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) s[k] = pk_add_sat(lab, v[k]);
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    if (m & (1u << r)) {
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[r][k] = pk_min(acc[r][k], s[k]);
    }
  }
}

// One wave per (block of 16 rows, 512-column panel); lanes own 8 columns
// (8 bytes of each gathered row); blocks by decreasing entry count; two
// rounds of U gathers in flight.  Rows of X and Y are read and written as
// whole 8-byte chunks (ldx, ldy multiples of 8, at least ncols rounded up).
template <int U>
__global__ void __launch_bounds__(256) compact_step_kernel(
    int64_t N, const int64_t *__restrict__ bptr, const uint64_t *__restrict__ ent,
    const int32_t *__restrict__ border, const uint8_t *__restrict__ X, int64_t ldx,
    const int32_t *__restrict__ RX, uint8_t *__restrict__ Y, int64_t ldy,
    const int32_t *__restrict__ RY, int64_t ncols, int32_t *__restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t groups = (nblocks + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t bslot = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (bslot >= nblocks) return;
  const int64_t b = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  const int64_t c0 = (panel * 64 + lane) * 8;
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;
  const kconst_i32 rx = (kconst_i32)RX;
  const kconst_i32 ry = (kconst_i32)RY;
  const gconst<u32x2> Xg = (gconst<u32x2>)to_global(X);
  const int64_t ld8 = ldx / 8;
  // lanes past the last column read chunk 0 of each row and store nothing
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / 8) : 0u;

  int32_t base = kDead;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q < N) base = min(base, ry[q]);
  }

  u16x2 acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[r][k] = splat(0xFFFFu);

  const int64_t e0 = bp[b], e1 = bp[b + 1];
  if (base < kDead && e0 < e1) {
    const int64_t last = e1 - 1;
    // per entry: mz = label z_p in bits 0..7, row mask in bits 8..23
    auto fetch = [&](int64_t i, uint32_t (&w)[U], int32_t (&o)[U], u32x2 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = i + u;
        const uint64_t x = en[k < last ? k : last];
        const uint32_t mz = (uint32_t)(x >> 24);
        w[u] = k <= last ? mz : (mz & 0xFFu);  // past the end: no rows
        const int64_t p = (int64_t)(uint32_t)(x & 0xFFFFFFu);
        o[u] = rx[p];
        v[u] = Xg[p * ld8 + off];
      }
    };
    auto apply = [&](const uint32_t (&w)[U], const int32_t (&o)[U], const u32x2 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // z_p + R_X[p] - base >= 0 for every successor of the block's rows
        const int32_t sh = o[u] + (int32_t)(w[u] & 0xFFu) - base;
        const uint16_t lab = (o[u] >= kDead || sh > 0xFFFF) ? (uint16_t)0xFFFFu : (uint16_t)sh;
        u16x2 row[4];
        unpack8(v[u].x, row[0], row[1]);
        unpack8(v[u].y, row[2], row[3]);
        apply_entry(acc, w[u] >> 8, splat(lab), row);
      }
    };
    uint32_t wa[U], wb[U];
    int32_t oa[U], ob[U];
    u32x2 va[U], vb[U];
    fetch(e0, wa, oa, va);
    for (int64_t i = e0;;) {
      bool more = i + U <= last;
      if (more) fetch(i + U, wb, ob, vb);
      apply(wa, oa, va);
      i += U;
      if (!more) break;
      more = i + U <= last;
      if (more) fetch(i + U, wa, oa, va);
      apply(wb, ob, vb);
      i += U;
      if (!more) break;
    }
  }
  if (c0 >= ncols) return;
  uint32_t bad = 0;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N) break;
    // (a vector load: the block's 16 offsets are not kept in scalar
    // registers across the gather loop)
    const int32_t rq = to_global(RY)[q];
    uint32_t lo, hi;
    if (rq >= kDead) {
      lo = hi = 0xFFFFFFFFu;
    } else {
      const int32_t gap = rq - base;
      if (gap > kMaxGap) bad = 1;
      const u16x2 d = splat((uint16_t)min(gap, 0xFFFF));
      u16x2 y[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) y[k] = __builtin_elementwise_sub_sat(acc[r][k], d);
      // residuals above 254 (not possible from held inputs) are reported
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (c0 + 2 * k < ncols && y[k].x > 254) bad = 1;
        if (c0 + 2 * k + 1 < ncols && y[k].y > 254) bad = 1;
      }
      lo = __builtin_amdgcn_perm(as_u32(y[1]), as_u32(y[0]), 0x06040200u);
      hi = __builtin_amdgcn_perm(as_u32(y[3]), as_u32(y[2]), 0x06040200u);
    }
    if (c0 + 8 <= ncols) {
      *(gmut<u32x2>)(to_global_mut(Y) + q * ldy + c0) = u32x2{lo, hi};
    } else {
      const gmut<uint8_t> yp = to_global_mut(Y) + q * ldy + c0;
      for (int k = 0; k < 8 && c0 + k < ncols; ++k)
        yp[k] = (uint8_t)(((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xFFu);
    }
  }
  if (bad) atomicOr(status, kStatusRange);
}

// One workgroup (256 lanes) per row: R = least entry, x = entry - R.
__global__ void __launch_bounds__(256) compact_from_u16_kernel(int64_t ncols, const uint16_t *X,
                                                               int64_t ldx, uint8_t *Y,
                                                               int64_t ldy, int32_t *R,
                                                               int32_t *status) {
  __shared__ int32_t red[3][4];
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const gconst<uint16_t> x = to_global(X) + q * ldx;
  int32_t mn = 0xFFFF, mx = -1, inf = 0;
  for (int64_t c = threadIdx.x; c < ncols; c += 256) {
    const int32_t v = x[c];
    mn = min(mn, v);
    if (v == 0xFFFF) inf = 1;
    else mx = max(mx, v);
  }
  mn = wave_min_i32(mn);
  mx = wave_max_i32(mx);
  inf = wave_max_i32(inf);
  if (lane == 0) {
    red[0][wv] = mn;
    red[1][wv] = mx;
    red[2][wv] = inf;
  }
  __syncthreads();
  mn = min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3]));
  mx = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
  inf = max(max(red[2][0], red[2][1]), max(red[2][2], red[2][3]));
  const bool dead = (mn == 0xFFFF);
  if (threadIdx.x == 0) {
    R[q] = dead ? kDead : mn;
    int32_t st = 0;
    if (!dead && inf) st |= kStatusMixed;
    if (!dead && mx - mn > 254) st |= kStatusRange;
    if (st) atomicOr(status, st);
  }
  const gmut<uint8_t> y = to_global_mut(Y) + q * ldy;
  for (int64_t c = threadIdx.x; c < ncols; c += 256) {
    const int32_t v = x[c];
    y[c] = (dead || v == 0xFFFF) ? (uint8_t)0xFF : (uint8_t)min(v - mn, 255);
  }
}

// P[q][c] = R[q] + x[q][c] saturated at INF = 65535 (x = 255 is INF).
__global__ void __launch_bounds__(256) compact_to_u16_kernel(int64_t ncols, const uint8_t *X,
                                                             int64_t ldx, const int32_t *R,
                                                             uint16_t *Y, int64_t ldy) {
  const int64_t q = blockIdx.x;
  const int32_t r = R[q];
  const gconst<uint8_t> x = to_global(X) + q * ldx;
  const gmut<uint16_t> y = to_global_mut(Y) + q * ldy;
  for (int64_t c = (int64_t)blockIdx.y * 256 + threadIdx.x; c < ncols;
       c += (int64_t)gridDim.y * 256) {
    const int32_t v = x[c];
    y[c] = (r >= kDead || v == 0xFF) ? (uint16_t)0xFFFFu : (uint16_t)min(r + v, 0xFFFF);
  }
}

// out = min(*out, min over live rows q of R[q] + x[q][q]) (entries past 65535
// count as INF = 65535).
__global__ void __launch_bounds__(256) compact_diag_kernel(int64_t N, const uint8_t *X,
                                                           int64_t ldx, const int32_t *R,
                                                           int32_t *out) {
  __shared__ int32_t red[4];
  int32_t m = 0xFFFF;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < N; q += (int64_t)gridDim.x * 256) {
    const int32_t r = R[q];
    const int32_t v = X[q * ldx + q];
    if (r < kDead && v != 0xFF) m = min(m, min(r + v, 0xFFFF));
  }
  m = wave_min_i32(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = min(min(red[0], red[1]), min(red[2], red[3]));
    if (m < 0xFFFF) atomicMin(out, m);
  }
}

// ---------------------------------------------------------------------------
// Shared-base form: one base G per power, P[q][c] = G + x[q][c], x in 0..254,
// every entry finite.  A whole power of A(D_n) spans a few units more than a
// row does, so it fits as well, and the step needs no per-entry offset: the
// label added per block entry is z_p as in the 16-bit step.  base[0] = G and
// base[1] = the least residual held.  The step writes its output relative to
// G_Y = G_X + base_X[1] (the least entry of the input: no entry of the output
// is below it, labels being non-negative), so output residuals are
// P_Y - min P_X: the span of the output plus the growth of its least entry.

// base_Y = {G_X + m_X, INT_MAX}; the step folds its least residual into [1].
__global__ void shared_prepare_kernel(const int32_t *bx, int32_t *by) {
  if (threadIdx.x == 0) {
    by[0] = bx[0] + bx[1];
    by[1] = 0x7FFFFFFF;
  }
}

// GROUPED: the block's entries a mask group at a time (the layout of
// blockstep.hip): each entry's z_p + x[p] goes into one group minimum (4
// packed mins per lane, no row tests) and the flagged last entry of a group
// applies it to the rows of its mask.  At n = 12 the 5.2e6 block entries
// form 8.2e4 groups, so the row tests and branches, which bound the kernel
// entry at a time on the scalar unit, run once per 64 entries.
template <int U, bool GROUPED>
__global__ void __launch_bounds__(256) shared_step_kernel(
    int64_t N, const int64_t *__restrict__ bptr, const uint64_t *__restrict__ ent,
    const int32_t *__restrict__ border, const uint8_t *__restrict__ X, int64_t ldx,
    const int32_t *__restrict__ bx, uint8_t *__restrict__ Y, int64_t ldy, int32_t *__restrict__ by,
    int64_t ncols, int32_t *__restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t groups = (nblocks + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t bslot = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (bslot >= nblocks) return;
  const int64_t b = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  const int64_t c0 = (panel * 64 + lane) * 8;
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;
  const gconst<u32x2> Xg = (gconst<u32x2>)to_global(X);
  const int64_t ld8 = ldx / 8;
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / 8) : 0u;

  u16x2 acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[r][k] = splat(0xFFFFu);
  u16x2 g[4] = {splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu)};

  const int64_t e0 = bp[b], e1 = bp[b + 1];
  if (e0 < e1) {
    // entry indices in 32 bits; a round inside the block is one scalar load
    // of U consecutive entries, only the last round clamps
    const uint32_t first = (uint32_t)e0, last = (uint32_t)(e1 - 1);
    typedef uint64_t round_t __attribute__((ext_vector_type(U), aligned(8)));
    auto fetch = [&](uint32_t i, uint64_t (&w)[U], u32x2 (&v)[U]) {
      if (i + (U - 1) <= last) {
        const round_t r = *(const __attribute__((address_space(4))) round_t *)(en + i);
#pragma unroll
        for (int u = 0; u < U; ++u) w[u] = r[u];
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint32_t k = i + u;
          const uint64_t x = en[min(k, last)];
          // past the end: no rows and no group end (the last entry's group
          // was applied, so what it adds to the group minimum is never used)
          w[u] = k <= last ? x : (x & 0xFFFFFFFFull);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = Xg[(int64_t)(uint32_t)(w[u] & 0xFFFFFFu) * ld8 + off];
    };
    auto apply = [&](const uint64_t (&w)[U], const u32x2 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        u16x2 row[4];
        unpack8(v[u].x, row[0], row[1]);
        unpack8(v[u].y, row[2], row[3]);
        const u16x2 lab = splat((uint16_t)((w[u] >> 24) & 0xFFu));
        if constexpr (GROUPED) {
#pragma unroll
          for (int k = 0; k < 4; ++k) g[k] = pk_min(g[k], pk_add_sat(lab, row[k]));
          if (w[u] & kGroupEnd) {
            const uint32_t m = (uint32_t)(w[u] >> 32);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
              if (m & (1u << r)) {
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[r][k] = pk_min(acc[r][k], g[k]);
              }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) g[k] = splat(0xFFFFu);
          }
        } else {
          apply_entry(acc, (uint32_t)(w[u] >> 32), lab, row);
        }
      }
    };
    uint64_t wa[U], wb[U];
    u32x2 va[U], vb[U];
    fetch(first, wa, va);
    for (uint32_t i = first;;) {
      bool more = i + U <= last;
      if (more) fetch(i + U, wb, vb);
      apply(wa, va);
      i += U;
      if (!more) break;
      more = i + U <= last;
      if (more) fetch(i + U, wa, va);
      apply(wb, vb);
      i += U;
      if (!more) break;
    }
  }
  const u16x2 d = splat((uint16_t)min(((kconst_i32)bx)[1], 0xFFFF));
  uint32_t bad = 0, low = 0xFFFFu;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N || c0 >= ncols) break;
    u16x2 y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) y[k] = __builtin_elementwise_sub_sat(acc[r][k], d);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (c0 + 2 * k < ncols) {
        bad |= (y[k].x > 254);
        low = min(low, (uint32_t)y[k].x);
      }
      if (c0 + 2 * k + 1 < ncols) {
        bad |= (y[k].y > 254);
        low = min(low, (uint32_t)y[k].y);
      }
    }
    const uint32_t lo = __builtin_amdgcn_perm(as_u32(y[1]), as_u32(y[0]), 0x06040200u);
    const uint32_t hi = __builtin_amdgcn_perm(as_u32(y[3]), as_u32(y[2]), 0x06040200u);
    if (c0 + 8 <= ncols) {
      *(gmut<u32x2>)(to_global_mut(Y) + q * ldy + c0) = u32x2{lo, hi};
    } else {
      const gmut<uint8_t> yp = to_global_mut(Y) + q * ldy + c0;
      for (int k = 0; k < 8 && c0 + k < ncols; ++k)
        yp[k] = (uint8_t)(((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xFFu);
    }
  }
  if (bad) atomicOr(status, kStatusRange);
  // one atomic per wave, and only when it lowers what is there (a stale read
  // can only add an atomic, never skip a needed one)
  const int32_t wlow = wave_min_i32((int32_t)low);
  if (lane == 0 && wlow < *(volatile int32_t *)(by + 1)) atomicMin(by + 1, wlow);
}

// base[0] = min(base[0], least entry); entries of INF are reported.
__global__ void __launch_bounds__(256) shared_min_kernel(int64_t ncols, const uint16_t *X,
                                                         int64_t ldx, int32_t *base,
                                                         int32_t *status) {
  __shared__ int32_t red[2][4];
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const gconst<uint16_t> x = to_global(X) + q * ldx;
  int32_t mn = 0xFFFF, inf = 0;
  for (int64_t c = threadIdx.x; c < ncols; c += 256) {
    const int32_t v = x[c];
    mn = min(mn, v);
    inf |= (v == 0xFFFF);
  }
  mn = wave_min_i32(mn);
  inf = wave_max_i32(inf);
  if (lane == 0) {
    red[0][wv] = mn;
    red[1][wv] = inf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mn = min(min(red[0][0], red[0][1]), min(red[0][2], red[0][3]));
    inf = max(max(red[1][0], red[1][1]), max(red[1][2], red[1][3]));
    atomicMin(base, mn);
    if (inf) atomicOr(status, kStatusMixed);
  }
}

// x = entry - base[0]; residuals above 254 are reported.
__global__ void __launch_bounds__(256) shared_residual_kernel(int64_t ncols, const uint16_t *X,
                                                              int64_t ldx, const int32_t *base,
                                                              uint8_t *Y, int64_t ldy,
                                                              int32_t *status) {
  const int64_t q = blockIdx.x;
  const int32_t g = base[0];
  const gconst<uint16_t> x = to_global(X) + q * ldx;
  const gmut<uint8_t> y = to_global_mut(Y) + q * ldy;
  int32_t bad = 0;
  for (int64_t c = threadIdx.x; c < ncols; c += 256) {
    const int32_t v = x[c] - g;
    bad |= (v > 254);
    y[c] = (uint8_t)min(v, 255);
  }
  if (bad) atomicOr(status, kStatusRange);
}

__global__ void __launch_bounds__(256) shared_to_u16_kernel(int64_t ncols, const uint8_t *X,
                                                            int64_t ldx, const int32_t *base,
                                                            uint16_t *Y, int64_t ldy) {
  const int64_t q = blockIdx.x;
  const int32_t g = base[0];
  const gconst<uint8_t> x = to_global(X) + q * ldx;
  const gmut<uint16_t> y = to_global_mut(Y) + q * ldy;
  for (int64_t c = (int64_t)blockIdx.y * 256 + threadIdx.x; c < ncols;
       c += (int64_t)gridDim.y * 256) {
    const int32_t v = x[c];
    y[c] = v == 0xFF ? (uint16_t)0xFFFFu : (uint16_t)min(g + v, 0xFFFF);
  }
}

__global__ void __launch_bounds__(256) shared_diag_kernel(int64_t N, const uint8_t *X,
                                                          int64_t ldx, const int32_t *base,
                                                          int32_t *out) {
  __shared__ int32_t red[4];
  const int32_t g = base[0];
  int32_t m = 0xFFFF;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < N; q += (int64_t)gridDim.x * 256) {
    const int32_t v = X[q * ldx + q];
    if (v != 0xFF) m = min(m, min(g + v, 0xFFFF));
  }
  m = wave_min_i32(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = min(min(red[0], red[1]), min(red[2], red[3]));
    if (m < 0xFFFF) atomicMin(out, m);
  }
}

// Trace of a product of two shared-base powers over selected diagonal
// entries (Theorem 2 with start states restricted to a list):
//   out = min(65535, G_X + G_P + min over t < count, k < N of x[r_t][k] + p[k][t])
// with r_t = idx[t] (or t without a list).  X supplies the rows r_t (count x N
// bytes read), P is an N x count panel (its column t belongs to state r_t).
// A workgroup takes 64 values of t and a run of 64-row k tiles; per tile each
// thread loads 16 bytes of one P row and 16 bytes of one X row, the X tile is
// stored transposed in LDS (k-major), and each thread folds its P row segment
// against the matching 16 bytes of LDS.  Byte arithmetic in 32-bit lanes.
constexpr int kTT = 64;          // t per workgroup
constexpr int kTK = 64;          // k per tile
constexpr int kXsRow = kTT + 16; // LDS row (bytes) of the transposed X tile: padded, 16-aligned

template <bool VEC>
__global__ void __launch_bounds__(256) shared_select_trace_kernel(
    int64_t N, int64_t count, const int32_t *__restrict__ idx, const uint8_t *__restrict__ X,
    int64_t ldx, const int32_t *__restrict__ bx, const uint8_t *__restrict__ P, int64_t ldp,
    const int32_t *__restrict__ bp, int64_t ktiles_per_wg, int32_t *out) {
  __shared__ __attribute__((aligned(16))) uint8_t xs[kTK][kXsRow];
  __shared__ int32_t red[4];
  const int tid = threadIdx.x;
  const int row = tid >> 2;         // k row of the P load; t row of the X load
  const int q = (tid & 3) * 16;     // 16-byte quarter of the row
  const int64_t t0 = (int64_t)blockIdx.x * kTT;
  const int64_t ktiles = (N + kTK - 1) / kTK;
  const int64_t kt_begin = (int64_t)blockIdx.y * ktiles_per_wg;
  const int64_t kt_end = min(ktiles, kt_begin + ktiles_per_wg);
  // the X row this thread loads: state r of t = t0 + row
  const int64_t tx = t0 + row;
  const bool tx_ok = tx < count;
  const int64_t r = tx_ok ? (idx ? (int64_t)idx[tx] : tx) : 0;
  const uint8_t *xrow = X + r * ldx;
  int32_t best = 0x7FFFFFFF;
  for (int64_t kt = kt_begin; kt < kt_end; ++kt) {
    const int64_t k0 = kt * kTK;
    // X tile: xs[k][t] = x[r_t][k0 + k]; 0xFF marks positions outside the matrix
    uint8_t xv[16];
    if (VEC && tx_ok && k0 + q < N) {
      const uint4 w = *(const uint4 *)(xrow + k0 + q);
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int i = 0; i < 16; ++i) xv[i] = (uint8_t)(ws[i >> 2] >> (8 * (i & 3)));
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        xv[i] = (tx_ok && k0 + q + i < N) ? xrow[k0 + q + i] : (uint8_t)0xFF;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) xs[q + i][row] = xv[i];
    // P tile row k0 + row, t0 + q .. t0 + q + 15
    const int64_t kp = k0 + row;
    uint32_t pw[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    if (kp < N) {
      const uint8_t *prow = P + kp * ldp + t0 + q;
      if (VEC && t0 + q < count) {
        const uint4 w = *(const uint4 *)prow;
        pw[0] = w.x;
        pw[1] = w.y;
        pw[2] = w.z;
        pw[3] = w.w;
      } else {
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (t0 + q + i < count)
            pw[i >> 2] = (pw[i >> 2] & ~(0xFFu << (8 * (i & 3)))) |
                         ((uint32_t)prow[i] << (8 * (i & 3)));
      }
    }
    __syncthreads();
    // fold: t = t0 + q + i, k = k0 + row; an entry is live when both sides
    // lie inside the matrices (t < count, k < N: checked, not inferred from 0xFF,
    // which a residual never takes but padding does)
    if (kp < N) {
      const uint4 w = *(const uint4 *)&xs[row][q];
      const uint32_t xw[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        if (t0 + q + i < count) {
          const int32_t a = (int32_t)((xw[i >> 2] >> (8 * (i & 3))) & 0xFFu);
          const int32_t b = (int32_t)((pw[i >> 2] >> (8 * (i & 3))) & 0xFFu);
          best = min(best, a + b);
        }
      }
    }
    __syncthreads();
  }
  best = wave_min_i32(best);
  if ((tid & 63) == 0) red[tid >> 6] = best;
  __syncthreads();
  if (tid == 0) {
    best = min(min(red[0], red[1]), min(red[2], red[3]));
    if (best != 0x7FFFFFFF) {
      const int64_t v = (int64_t)bx[0] + (int64_t)bp[0] + best;
      atomicMin(out, (int32_t)min<int64_t>(v, 0xFFFF));
    }
  }
}

bool chunk_ok(const void *p, int64_t ld, int64_t ncols) {
  return ((uintptr_t)p % 8 == 0) && (ld % 8 == 0) && ld >= (ncols + 7) / 8 * 8;
}

}  // namespace

std::atomic<int> g_compact_chain_from{11};

bool compact_chain(int n) {
  const int from = g_compact_chain_from.load();
  return from > 0 && n >= from;
}

hipError_t launch_shared_from_u16(int64_t N, int64_t ncols, const uint16_t *X, int64_t ldx,
                                  uint8_t *Y, int64_t ldy, int32_t *base, int32_t *status,
                                  hipStream_t s) {
  hipError_t e = launch_fill_i32(base, 1, 0xFFFF, s);
  if (e == hipSuccess) e = launch_fill_i32(base + 1, 1, 0, s);
  if (e != hipSuccess || N == 0 || ncols == 0) return e;
  hipLaunchKernelGGL(shared_min_kernel, dim3((unsigned)N), dim3(256), 0, s, ncols, X, ldx, base,
                     status);
  hipLaunchKernelGGL(shared_residual_kernel, dim3((unsigned)N), dim3(256), 0, s, ncols, X, ldx,
                     (const int32_t *)base, Y, ldy, status);
  return hipGetLastError();
}

hipError_t launch_shared_to_u16(int64_t N, int64_t ncols, const uint8_t *X, int64_t ldx,
                                const int32_t *base, uint16_t *Y, int64_t ldy, hipStream_t s) {
  if (N == 0 || ncols == 0) return hipSuccess;
  const dim3 grid((unsigned)N, (unsigned)std::min<int64_t>((ncols + 255) / 256, 64));
  hipLaunchKernelGGL(shared_to_u16_kernel, grid, dim3(256), 0, s, ncols, X, ldx, base, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_shared_step(const StateView &v, const uint8_t *X, int64_t ldx, const int32_t *bx,
                              uint8_t *Y, int64_t ldy, int32_t *by, int64_t ncols,
                              int32_t *status, hipStream_t s) {
  const int64_t N = v.N;
  hipLaunchKernelGGL(shared_prepare_kernel, dim3(1), dim3(64), 0, s, bx, by);
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t panels = (ncols + 511) / 512;
  const dim3 grid((unsigned)(((nblocks + 3) / 4) * panels));
  const bool grouped = g_grouped != 0, eight = g_unroll == 8;
  if (grouped && eight)
    hipLaunchKernelGGL((shared_step_kernel<8, true>), grid, dim3(256), 0, s, N, v.bptr, v.bent,
                       v.border, X, ldx, bx, Y, ldy, by, ncols, status);
  else if (grouped)
    hipLaunchKernelGGL((shared_step_kernel<4, true>), grid, dim3(256), 0, s, N, v.bptr, v.bent,
                       v.border, X, ldx, bx, Y, ldy, by, ncols, status);
  else if (eight)
    hipLaunchKernelGGL((shared_step_kernel<8, false>), grid, dim3(256), 0, s, N, v.bptr, v.bent,
                       v.border, X, ldx, bx, Y, ldy, by, ncols, status);
  else
    hipLaunchKernelGGL((shared_step_kernel<4, false>), grid, dim3(256), 0, s, N, v.bptr, v.bent,
                       v.border, X, ldx, bx, Y, ldy, by, ncols, status);
  return hipGetLastError();
}

hipError_t launch_shared_diag(int64_t N, const uint8_t *X, int64_t ldx, const int32_t *base,
                              int32_t *out, hipStream_t s) {
  hipError_t e = launch_fill_i32(out, 1, 0xFFFF, s);
  if (e != hipSuccess || N == 0) return e;
  const unsigned blocks = (unsigned)std::min<int64_t>((N + 255) / 256, 1024);
  hipLaunchKernelGGL(shared_diag_kernel, dim3(blocks), dim3(256), 0, s, N, X, ldx, base, out);
  return hipGetLastError();
}

hipError_t launch_shared_select_trace(int64_t N, int64_t count, const int32_t *idx,
                                      const uint8_t *X, int64_t ldx, const int32_t *bx,
                                      const uint8_t *P, int64_t ldp, const int32_t *bp,
                                      int32_t *out, hipStream_t s) {
  hipError_t e = launch_fill_i32(out, 1, 0xFFFF, s);
  if (e != hipSuccess || N == 0 || count == 0) return e;
  const int64_t ttiles = (count + kTT - 1) / kTT;
  const int64_t ktiles = (N + kTK - 1) / kTK;
  // about 4096 workgroups over the t tiles and runs of k tiles
  const int64_t ysplit = std::max<int64_t>(1, std::min<int64_t>(ktiles, 4096 / ttiles));
  const int64_t per = (ktiles + ysplit - 1) / ysplit;
  const dim3 grid((unsigned)ttiles, (unsigned)((ktiles + per - 1) / per));
  const bool vec = ((uintptr_t)X % 16 == 0) && ((uintptr_t)P % 16 == 0) && ldx % 16 == 0 &&
                   ldp % 16 == 0;
  if (vec)
    hipLaunchKernelGGL(shared_select_trace_kernel<true>, grid, dim3(256), 0, s, N, count, idx, X,
                       ldx, bx, P, ldp, bp, per, out);
  else
    hipLaunchKernelGGL(shared_select_trace_kernel<false>, grid, dim3(256), 0, s, N, count, idx,
                       X, ldx, bx, P, ldp, bp, per, out);
  return hipGetLastError();
}

}  // namespace tp

using namespace tp;

extern "C" {

int tp_compact_from_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx, void *d_Y,
                        int64_t ldy, int32_t *d_R, int32_t *d_status, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && ncols >= 0 && N < ((int64_t)1 << 31), "bad size");
  if (N == 0) return TP_OK;
  TP_REQUIRE(ldx >= (ncols > 0 ? ncols : 1) && ldy >= (ncols > 0 ? ncols : 1),
             "leading dimension < ncols");
  TP_REQUIRE(d_X && d_Y && d_R && d_status, "NULL pointer");
  hipLaunchKernelGGL(compact_from_u16_kernel, dim3((unsigned)N), dim3(256), 0, stream, ncols,
                     (const uint16_t *)d_X, ldx, (uint8_t *)d_Y, ldy, d_R, d_status);
  TP_HIP_CHECK(hipGetLastError());
  return TP_OK;
}

int tp_compact_to_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx, const int32_t *d_R,
                      void *d_Y, int64_t ldy, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && ncols >= 0 && N < ((int64_t)1 << 31), "bad size");
  if (N == 0 || ncols == 0) return TP_OK;
  TP_REQUIRE(ldx >= ncols && ldy >= ncols, "leading dimension < ncols");
  TP_REQUIRE(d_X && d_Y && d_R, "NULL pointer");
  const dim3 grid((unsigned)N, (unsigned)std::min<int64_t>((ncols + 255) / 256, 64));
  hipLaunchKernelGGL(compact_to_u16_kernel, grid, dim3(256), 0, stream, ncols,
                     (const uint8_t *)d_X, ldx, d_R, (uint16_t *)d_Y, ldy);
  TP_HIP_CHECK(hipGetLastError());
  return TP_OK;
}

int tp_compact_step(int n, const void *d_X, int64_t ldx, const int32_t *d_RX, void *d_Y,
                    int64_t ldy, int32_t *d_RY, int64_t ncols, int32_t *d_status,
                    hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(ncols >= 0, "negative size");
  if (ncols == 0) return TP_OK;
  TP_REQUIRE(d_X && d_Y && d_RX && d_RY && d_status, "NULL pointer");
  TP_REQUIRE(d_X != d_Y && d_RX != d_RY, "the step cannot run in place");
  TP_REQUIRE(chunk_ok(d_X, ldx, ncols) && chunk_ok(d_Y, ldy, ncols),
             "X and Y need 8-byte aligned rows with ld a multiple of 8, at least ncols "
             "rounded up to 8");
  StateView v;
  const int rc = state_view(n, stream, &v);
  if (rc != TP_OK) return rc;
  const int64_t N = v.N;
  hipLaunchKernelGGL(compact_offsets_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, stream,
                     N, v.rowptr, v.colz, d_RX, d_RY);
  TP_HIP_CHECK(hipGetLastError());
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t panels = (ncols + 511) / 512;
  const dim3 grid((unsigned)(((nblocks + 3) / 4) * panels));
  if (g_unroll == 8)
    hipLaunchKernelGGL((compact_step_kernel<8>), grid, dim3(256), 0, stream, N, v.bptr, v.bent,
                       v.border, (const uint8_t *)d_X, ldx, d_RX, (uint8_t *)d_Y, ldy,
                       (const int32_t *)d_RY, ncols, d_status);
  else
    hipLaunchKernelGGL((compact_step_kernel<4>), grid, dim3(256), 0, stream, N, v.bptr, v.bent,
                       v.border, (const uint8_t *)d_X, ldx, d_RX, (uint8_t *)d_Y, ldy,
                       (const int32_t *)d_RY, ncols, d_status);
  TP_HIP_CHECK(hipGetLastError());
  return TP_OK;
}

int tp_compact_diag_min(int64_t N, const void *d_X, int64_t ldx, const int32_t *d_R,
                        int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && N < ((int64_t)1 << 31), "bad size");
  TP_REQUIRE(d_out != nullptr, "out is NULL");
  TP_HIP_CHECK(launch_fill_i32(d_out, 1, 0xFFFF, stream));
  if (N == 0) return TP_OK;
  TP_REQUIRE(ldx >= N && d_X && d_R, "bad X or R");
  const unsigned blocks = (unsigned)std::min<int64_t>((N + 255) / 256, 1024);
  hipLaunchKernelGGL(compact_diag_kernel, dim3(blocks), dim3(256), 0, stream, N,
                     (const uint8_t *)d_X, ldx, d_R, d_out);
  TP_HIP_CHECK(hipGetLastError());
  return TP_OK;
}

int tp_compact_shared_from_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx,
                               void *d_Y, int64_t ldy, int32_t *d_base, int32_t *d_status,
                               hipStream_t stream) {
  TP_REQUIRE(N >= 0 && ncols >= 0 && N < ((int64_t)1 << 31), "bad size");
  TP_REQUIRE(d_base && d_status, "NULL pointer");
  TP_REQUIRE(N == 0 || ncols == 0 || (ldx >= ncols && ldy >= ncols && d_X && d_Y),
             "bad X or Y");
  TP_HIP_CHECK(launch_shared_from_u16(N, ncols, (const uint16_t *)d_X, ldx, (uint8_t *)d_Y, ldy,
                                      d_base, d_status, stream));
  return TP_OK;
}

int tp_compact_shared_to_u16(int64_t N, int64_t ncols, const void *d_X, int64_t ldx,
                             const int32_t *d_base, void *d_Y, int64_t ldy, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && ncols >= 0 && N < ((int64_t)1 << 31), "bad size");
  if (N == 0 || ncols == 0) return TP_OK;
  TP_REQUIRE(ldx >= ncols && ldy >= ncols, "leading dimension < ncols");
  TP_REQUIRE(d_X && d_Y && d_base, "NULL pointer");
  TP_HIP_CHECK(launch_shared_to_u16(N, ncols, (const uint8_t *)d_X, ldx, d_base, (uint16_t *)d_Y,
                                    ldy, stream));
  return TP_OK;
}

int tp_compact_shared_step(int n, const void *d_X, int64_t ldx, const int32_t *d_bx, void *d_Y,
                           int64_t ldy, int32_t *d_by, int64_t ncols, int32_t *d_status,
                           hipStream_t stream) {
  TP_REQUIRE(n >= 1 && n <= 13, "n = %d outside 1..13", n);
  TP_REQUIRE(ncols >= 0, "negative size");
  TP_REQUIRE(d_bx && d_by && d_bx != d_by, "base words NULL or shared");
  if (ncols == 0) return TP_OK;
  TP_REQUIRE(d_X && d_Y && d_status, "NULL pointer");
  TP_REQUIRE(d_X != d_Y, "the step cannot run in place");
  TP_REQUIRE(chunk_ok(d_X, ldx, ncols) && chunk_ok(d_Y, ldy, ncols),
             "X and Y need 8-byte aligned rows with ld a multiple of 8, at least ncols "
             "rounded up to 8");
  StateView v;
  const int rc = state_view(n, stream, &v);
  if (rc != TP_OK) return rc;
  TP_HIP_CHECK(launch_shared_step(v, (const uint8_t *)d_X, ldx, d_bx, (uint8_t *)d_Y, ldy, d_by,
                                  ncols, d_status, stream));
  return TP_OK;
}

int tp_compact_shared_diag_min(int64_t N, const void *d_X, int64_t ldx, const int32_t *d_base,
                               int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && N < ((int64_t)1 << 31), "bad size");
  TP_REQUIRE(d_out != nullptr, "out is NULL");
  TP_REQUIRE(N == 0 || (ldx >= N && d_X && d_base), "bad X or base");
  TP_HIP_CHECK(launch_shared_diag(N, (const uint8_t *)d_X, ldx, d_base, d_out, stream));
  return TP_OK;
}

int tp_compact_shared_select_trace(int64_t N, int64_t count, const int32_t *d_idx,
                                   const void *d_X, int64_t ldx, const int32_t *d_bx,
                                   const void *d_P, int64_t ldp, const int32_t *d_bp,
                                   int32_t *d_out, hipStream_t stream) {
  TP_REQUIRE(N >= 0 && count >= 0 && N < ((int64_t)1 << 31), "bad size");
  TP_REQUIRE(d_out != nullptr, "out is NULL");
  TP_REQUIRE(d_idx != nullptr || count <= N, "count %lld exceeds N %lld without a row list",
             (long long)count, (long long)N);
  TP_REQUIRE(N == 0 || count == 0 ||
                 (d_X && d_P && d_bx && d_bp && ldx >= N && ldp >= count),
             "bad X, P or base words");
  TP_HIP_CHECK(launch_shared_select_trace(N, count, d_idx, (const uint8_t *)d_X, ldx, d_bx,
                                          (const uint8_t *)d_P, ldp, d_bp, d_out, stream));
  return TP_OK;
}

int tp_tune_compact_chains(int compact_from_n) {
  TP_REQUIRE(compact_from_n >= 0, "negative path order");
  g_compact_chain_from = compact_from_n;
  return TP_OK;
}

int tp_tune_compact_step(int unroll) {
  const int u = unroll & ~TP_COMPACT_GROUPED;
  TP_REQUIRE(unroll == 0 || u == 4 || u == 8, "unroll %d is not 0, 4 or 8 (| TP_COMPACT_GROUPED)",
             unroll);
  g_unroll = unroll == 0 ? 8 : u;
  g_grouped = unroll == 0 || (unroll & TP_COMPACT_GROUPED) != 0;
  return TP_OK;
}

}  // extern "C"
