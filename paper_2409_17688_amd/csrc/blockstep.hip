// The sparse left step Y = A(D_n) x X in row blocks.
//
// Row q of the product is a gather: Y[q][j] = min over successors p of q of
// (z_p + X[p][j]) (the arc label z_p, the number of zeros of word p, depends
// on the successor only; Section 2.2).  Consecutive words differ only in
// their last letters, so consecutive rows share most successors: over 16
// consecutive rows of A(D_n), n = 8..10, the union of the successor lists is
// about a quarter of their total length.  This kernel walks that union once
// per block of 16 rows, so each gathered row of X is read once per block
// instead of once per row, and applies it to the rows of the block that have
// it as a successor (a 16-bit mask per entry).
//
// The blocked form of A(D_n): for block b (rows 16b .. 16b+15), entries
// bptr[b] .. bptr[b+1]-1, each a 64-bit word
//   bits  0..23  successor p        (N < 2^24 for n <= 12)
//   bits 24..31  its label z_p
//   bits 32..47  mask: bit r set when p is a successor of row 16b + r
//   bit  48      set on the last entry of a run with one mask
// It is built from the word masks with the same "can follow" test as the CSR
// (two passes: count, then fill in increasing p after a scan); the state
// cache then groups each block's entries by mask (by p within a group) and
// flags the last of each group, for the steps that take one minimum per
// group before touching the rows.
//
// Launch shape of the step: one wave per (block, 512-column panel); lanes own
// 8 consecutive columns; the 16 rows' accumulators live in registers (64
// packed registers); entries are read with scalar loads (they are uniform in
// the wave) and the per-row updates are skipped by uniform branches on the
// mask, so the arithmetic is that of the plain gather.  Workgroups are
// numbered so each XCD takes a contiguous range of blocks of one panel.
#include "device_core.hpp"

namespace tp {

namespace {

constexpr int kRows = 16;  // rows per block

// acc[r] = min(acc[r], g) for the rows r whose bit is set in m.
__device__ __forceinline__ void apply_group(u16x2 (&acc)[kRows][4], uint32_t m,
                                            const u16x2 (&g)[4]) {
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    if (m & (1u << r)) {
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[r][k] = pk_min(acc[r][k], g[k]);
    }
  }
}

// One wave per block: number of distinct successors of its rows.
__global__ void block_count_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                   int64_t *__restrict__ bptr) {
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (b >= nblocks) return;
  uint32_t mq[kRows];
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    mq[r] = q < N ? masks[q] : 0u;
  }
  const int rows = (int)std::min<int64_t>(kRows, N - b * kRows);
  int64_t cnt = 0;
  for (int64_t p0 = 0; p0 < N; p0 += 64) {
    const int64_t p = p0 + lane;
    bool arc = false;
    if (p < N) {
      const uint32_t mp = masks[p];
      for (int r = 0; r < rows && !arc; ++r) arc = can_follow(mq[r], mp, full);
    }
    cnt += __popcll(__ballot(arc));
  }
  if (lane == 0) {
    bptr[b + 1] = cnt;
    if (b == 0) bptr[0] = 0;
  }
}

// One wave per block: its entries in increasing p.
__global__ void block_fill_kernel(int64_t N, uint32_t full, const uint32_t *__restrict__ masks,
                                  const int64_t *__restrict__ bptr, uint64_t *__restrict__ ent) {
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t b = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (b >= nblocks) return;
  uint32_t mq[kRows];
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    mq[r] = q < N ? masks[q] : 0u;
  }
  const int rows = (int)std::min<int64_t>(kRows, N - b * kRows);
  int64_t pos = bptr[b];
  for (int64_t p0 = 0; p0 < N; p0 += 64) {
    const int64_t p = p0 + lane;
    uint32_t m = 0, mp = 0;
    if (p < N) {
      mp = masks[p];
      for (int r = 0; r < rows; ++r) m |= (uint32_t)can_follow(mq[r], mp, full) << r;
    }
    const uint64_t bal = __ballot(m != 0);
    if (m != 0) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      const uint32_t z = (uint32_t)__builtin_popcount(mp & 0xFFFFu);
      ent[pos + below] = ((uint64_t)m << 32) | ((uint64_t)z << 24) | (uint64_t)p;
    }
    pos += __popcll(bal);
  }
}

// acc[r] = min(acc[r], lab + v) for the rows r whose bit is set in m (m is
// wave-uniform: the skipped rows cost a scalar test and branch only).
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

// 16-bit entries only (the power chains run in u16).
template <bool VEC, int U>
__global__ void __launch_bounds__(256) block_step_kernel(int64_t N, const int64_t *__restrict__ bptr,
                                                         const uint64_t *__restrict__ ent,
                                                         const int32_t *__restrict__ border,
                                                         const uint16_t *__restrict__ X,
                                                         int64_t ldx, uint16_t *__restrict__ Y,
                                                         int64_t ldy, int64_t ncols) {
  using T = uint16_t;
  constexpr int VE = 8;
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t groups = (nblocks + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t bslot = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (bslot >= nblocks) return;
  // blocks with the most entries first
  const int64_t b = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  const int64_t c0 = (panel * 64 + lane) * VE;
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;

  u16x2 acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[r][k] = splat(0xFFFFu);

  const int64_t e0 = bp[b], e1 = bp[b + 1];
  int64_t i = e0;
  for (; i + U <= e1; i += U) {
    uint64_t w[U];
    u16x2 v[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      w[u] = en[i + u];
      load_row_chunk<T, VEC>(X, ldx, (int64_t)(uint32_t)(w[u] & 0xFFFFFFu), c0, ncols, v[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      apply_entry(acc, (uint32_t)(w[u] >> 32), splat((uint16_t)((w[u] >> 24) & 0xFFu)), v[u]);
  }
  for (; i < e1; ++i) {
    const uint64_t w = en[i];
    u16x2 v[4];
    load_row_chunk<T, VEC>(X, ldx, (int64_t)(uint32_t)(w & 0xFFFFFFu), c0, ncols, v);
    apply_entry(acc, (uint32_t)(w >> 32), splat((uint16_t)((w >> 24) & 0xFFu)), v);
  }
  if (c0 >= ncols) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N) break;
    T *yrow = Y + q * ldy + c0;
    const u16x2 *a = acc[r];
    if (VEC && c0 + VE <= ncols) {
      *reinterpret_cast<uint4 *>(yrow) = uint4{as_u32(a[0]), as_u32(a[1]), as_u32(a[2]),
                                               as_u32(a[3])};
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (c0 + 2 * k < ncols) yrow[2 * k] = (T)a[k].x;
        if (c0 + 2 * k + 1 < ncols) yrow[2 * k + 1] = (T)a[k].y;
      }
    }
  }
}

// The same step for 16-byte aligned rows at least ncols rounded up to 8 long
// (the library's own padded powers): rows are read as whole 16-byte chunks
// and the next U entries' rows are requested before the current U are
// applied, so two rounds of gathers are in flight.  A last partial round
// repeats the block's last entry with an empty row mask, which changes
// nothing.
//
// GROUPED: the entries are taken a mask group at a time (the layout above):
// each entry's z_p + X[p] goes into one group minimum, and the flagged last
// entry of a group applies that minimum to the rows of its mask, so the row
// tests run once per group instead of once per entry.
template <int U, bool GROUPED>
__global__ void __launch_bounds__(256) block_step_pipe_kernel(
    int64_t N, const int64_t *__restrict__ bptr, const uint64_t *__restrict__ ent,
    const int32_t *__restrict__ border, const uint16_t *__restrict__ X, int64_t ldx,
    uint16_t *__restrict__ Y, int64_t ldy, int64_t ncols) {
  const int lane = threadIdx.x & 63;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t groups = (nblocks + 3) / 4;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / groups;
  const int64_t bslot = (t - panel * groups) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (bslot >= nblocks) return;
  // blocks with the most entries first
  const int64_t b = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  const int64_t c0 = (panel * 64 + lane) * 8;
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;
  const gconst<u32x4> Xg = (gconst<u32x4>)to_global(X);
  const int64_t ld4 = ldx / 8;
  // lanes past the last column read chunk 0 of each row (inside the row) and
  // store nothing
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / 8) : 0u;

  u16x2 acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[r][k] = splat(0xFFFFu);
  u16x2 g[4] = {splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu)};

  const int64_t e0 = bp[b], e1 = bp[b + 1];
  if (e0 < e1) {
    const int64_t last = e1 - 1;
    auto fetch = [&](int64_t i, uint64_t (&w)[U], u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = i + u;
        const uint64_t x = en[k < last ? k : last];
        // past the end: no rows and no group end (the last entry's group was
        // applied, so what it adds to the group minimum is never used)
        w[u] = k <= last ? x : (x & 0xFFFFFFFFull);
        v[u] = Xg[(int64_t)(uint32_t)(x & 0xFFFFFFu) * ld4 + off];
      }
    };
    auto apply = [&](const uint64_t (&w)[U], const u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const u16x2 row[4] = {as_pk(v[u].x), as_pk(v[u].y), as_pk(v[u].z), as_pk(v[u].w)};
        const u16x2 lab = splat((uint16_t)((w[u] >> 24) & 0xFFu));
        if constexpr (GROUPED) {
#pragma unroll
          for (int k = 0; k < 4; ++k) g[k] = pk_min(g[k], pk_add_sat(lab, row[k]));
          if (w[u] & kGroupEnd) {
            apply_group(acc, (uint32_t)(w[u] >> 32), g);
#pragma unroll
            for (int k = 0; k < 4; ++k) g[k] = splat(0xFFFFu);
          }
        } else {
          apply_entry(acc, (uint32_t)(w[u] >> 32), lab, row);
        }
      }
    };
    uint64_t wa[U], wb[U];
    u32x4 va[U], vb[U];
    fetch(e0, wa, va);
    for (int64_t i = e0;;) {
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
  if (c0 >= ncols) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N) break;
    const u16x2 *a = acc[r];
    if (c0 + 8 <= ncols) {
      *(gmut<u32x4>)(to_global_mut(Y) + q * ldy + c0) =
          u32x4{as_u32(a[0]), as_u32(a[1]), as_u32(a[2]), as_u32(a[3])};
    } else {
      const gmut<uint16_t> y = to_global_mut(Y) + q * ldy + c0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (c0 + 2 * k < ncols) y[2 * k] = a[k].x;
        if (c0 + 2 * k + 1 < ncols) y[2 * k + 1] = a[k].y;
      }
    }
  }
}

// Small path orders: a block's entries split across the W waves of one
// workgroup (a run of at most ceil(E / W) of the E entries each, mask groups
// as above, the run's last entry closing its group), each wave folding its
// own minima for the block's 16 rows; the W partial minima meet in LDS (a
// tree: half the waves hand theirs to the other half each round) and wave 0
// stores the rows.  With one wave per block, n = 8 (87 blocks, 3
// panels of 512 columns) left most of the chip idle and made each block's
// whole entry list one chain of dependent gathers.
template <int U, int W>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(4)))
block_split_step_kernel(
    int64_t N, const int64_t *__restrict__ bptr, const uint64_t *__restrict__ ent,
    const int32_t *__restrict__ border, const uint16_t *__restrict__ X, int64_t ldx,
    uint16_t *__restrict__ Y, int64_t ldy, int64_t ncols) {
  __shared__ uint32_t part[W / 2][kRows * 4][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / nblocks;
  const int64_t bslot = t - panel * nblocks;
  const int64_t b = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  const int64_t c0 = (panel * 64 + lane) * 8;
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;
  const gconst<u32x4> Xg = (gconst<u32x4>)to_global(X);
  const int64_t ld4 = ldx / 8;
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / 8) : 0u;

  u16x2 acc[kRows][4];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[r][k] = splat(0xFFFFu);
  u16x2 g[4] = {splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu), splat(0xFFFFu)};

  const int64_t e0 = bp[b], e1 = bp[b + 1];
  const int64_t per = (e1 - e0 + W - 1) / W;
  const int64_t my0 = e0 + (int64_t)wave * per, my1 = min(e1, my0 + per);
  if (my0 < my1) {
    const int64_t last = my1 - 1;
    auto fetch = [&](int64_t i, uint64_t (&w)[U], u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = i + u;
        const uint64_t x = en[k < last ? k : last];
        // the run's last entry closes its group; past it: no rows, no group end
        w[u] = k < last ? x : (k == last ? (x | kGroupEnd) : (x & 0xFFFFFFFFull));
        v[u] = Xg[(int64_t)(uint32_t)(x & 0xFFFFFFu) * ld4 + off];
      }
    };
    auto apply = [&](const uint64_t (&w)[U], const u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const u16x2 lab = splat((uint16_t)((w[u] >> 24) & 0xFFu));
        g[0] = pk_min(g[0], pk_add_sat(lab, as_pk(v[u].x)));
        g[1] = pk_min(g[1], pk_add_sat(lab, as_pk(v[u].y)));
        g[2] = pk_min(g[2], pk_add_sat(lab, as_pk(v[u].z)));
        g[3] = pk_min(g[3], pk_add_sat(lab, as_pk(v[u].w)));
        if (w[u] & kGroupEnd) {
          apply_group(acc, (uint32_t)(w[u] >> 32), g);
#pragma unroll
          for (int k = 0; k < 4; ++k) g[k] = splat(0xFFFFu);
        }
      }
    };
    uint64_t wa[U], wb[U];
    u32x4 va[U], vb[U];
    fetch(my0, wa, va);
    for (int64_t i = my0;;) {
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
  // the W partial minima meet in LDS, halving the waves each round
#pragma unroll 1
  for (int half = W / 2; half >= 1; half /= 2) {
    if (wave >= half && wave < 2 * half) {
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k) part[wave - half][r * 4 + k][lane] = as_u32(acc[r][k]);
    }
    __syncthreads();
    if (wave < half) {
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          acc[r][k] = pk_min(acc[r][k], as_pk(part[wave][r * 4 + k][lane]));
    }
    __syncthreads();
  }
  if (wave != 0 || c0 >= ncols) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N) break;
    const u16x2 *a = acc[r];
    if (c0 + 8 <= ncols) {
      *(gmut<u32x4>)(to_global_mut(Y) + q * ldy + c0) =
          u32x4{as_u32(a[0]), as_u32(a[1]), as_u32(a[2]), as_u32(a[3])};
    } else {
      const gmut<uint16_t> y = to_global_mut(Y) + q * ldy + c0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (c0 + 2 * k < ncols) y[2 * k] = a[k].x;
        if (c0 + 2 * k + 1 < ncols) y[2 * k + 1] = a[k].y;
      }
    }
  }
}

hipError_t launch_block_step_u16(int64_t N, const int64_t *bptr, const uint64_t *ent,
                                 const int32_t *border, const uint16_t *X, int64_t ldx,
                                 uint16_t *Y, int64_t ldy, int64_t ncols, bool grouped,
                                 hipStream_t s) {
  constexpr int VE = 8;
  const int64_t nblocks = (N + kRows - 1) / kRows;
  const int64_t panels = (ncols + 64 * VE - 1) / (64 * VE);
  const dim3 grid((unsigned)(((nblocks + 3) / 4) * panels));
  const bool vec = (ldx % VE == 0) && (ldy % VE == 0) && ((uintptr_t)X % 16 == 0) &&
                   ((uintptr_t)Y % 16 == 0);
  // the pipelined kernel (two rounds of gathers in flight) wherever rows can
  // be read as whole 16-byte chunks: with the blocks taken longest first it
  // is as fast as the plain one at n = 12 (45.6 ms) and faster below (n = 11:
  // 5.41 vs 5.58 ms; n = 9: 0.30 vs 0.52 ms)
  // grouped, on 16-byte rows: one wave per (block, panel) where that fills
  // the chip; below that a workgroup of 8 or 4 waves shares each block
  const int64_t items = nblocks * panels;
  const bool pipe_ok = vec && ldx >= (ncols + 7) / 8 * 8;
  if (pipe_ok && grouped && items < 1024)
    hipLaunchKernelGGL((block_split_step_kernel<4, 16>), dim3((unsigned)items), dim3(1024), 0, s,
                       N, bptr, ent, border, X, ldx, Y, ldy, ncols);
  else if (pipe_ok && grouped && items < 4096)
    hipLaunchKernelGGL((block_split_step_kernel<4, 8>), dim3((unsigned)items), dim3(512), 0, s,
                       N, bptr, ent, border, X, ldx, Y, ldy, ncols);
  else if (pipe_ok && grouped)
    hipLaunchKernelGGL((block_step_pipe_kernel<8, true>), grid, dim3(256), 0, s, N, bptr, ent,
                       border, X, ldx, Y, ldy, ncols);
  else if (pipe_ok)
    hipLaunchKernelGGL((block_step_pipe_kernel<4, false>), grid, dim3(256), 0, s, N, bptr, ent,
                       border, X, ldx, Y, ldy, ncols);
  else if (vec)
    hipLaunchKernelGGL((block_step_kernel<true, 4>), grid, dim3(256), 0, s, N, bptr, ent, border,
                       X, ldx, Y, ldy, ncols);
  else
    hipLaunchKernelGGL((block_step_kernel<false, 4>), grid, dim3(256), 0, s, N, bptr, ent,
                       border, X, ldx, Y, ldy, ncols);
  return hipGetLastError();
}

}  // namespace

int64_t block_count_host(int64_t N) { return (N + kRows - 1) / kRows; }

hipError_t launch_block_count(int64_t N, int n, const uint32_t *masks, int64_t *bptr,
                              hipStream_t s) {
  if (N == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int64_t nb = block_count_host(N);
  hipLaunchKernelGGL(block_count_kernel, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, N, full,
                     masks, bptr);
  return hipGetLastError();
}

hipError_t launch_block_fill(int64_t N, int n, const uint32_t *masks, const int64_t *bptr,
                             uint64_t *ent, hipStream_t s) {
  if (N == 0) return hipSuccess;
  const uint32_t full = (1u << n) - 1u;
  const int64_t nb = block_count_host(N);
  hipLaunchKernelGGL(block_fill_kernel, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, N, full,
                     masks, bptr, ent);
  return hipGetLastError();
}

hipError_t launch_block_step(int64_t N, const int64_t *bptr, const uint64_t *ent,
                             const int32_t *border, const uint16_t *X, int64_t ldx, uint16_t *Y,
                             int64_t ldy, int64_t ncols, bool grouped, hipStream_t s) {
  if (N == 0 || ncols == 0) return hipSuccess;
  return launch_block_step_u16(N, bptr, ent, border, X, ldx, Y, ldy, ncols, grouped, s);
}

}  // namespace tp
