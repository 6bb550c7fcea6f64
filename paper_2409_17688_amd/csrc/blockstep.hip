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

constexpr int kRows = kBlockRows;  // rows per block

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
    // entry indices in 32 bits; a round inside the block is one scalar load
    // of U consecutive entries, only the last round clamps
    const uint32_t first = (uint32_t)e0, last = (uint32_t)(e1 - 1);
    typedef uint64_t round_t __attribute__((ext_vector_type(U), aligned(8)));
    auto fetch = [&](uint32_t i, uint64_t (&w)[U], u32x4 (&v)[U]) {
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
      for (int u = 0; u < U; ++u) v[u] = Xg[(int64_t)(uint32_t)(w[u] & 0xFFFFFFu) * ld4 + off];
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
// own minima for the block's 16 rows at its lane's 2V columns; the W partial
// minima meet in LDS (a tree: half the waves hand theirs to the other half
// each round) and wave 0 stores the rows.  With one wave per block, n = 8 (87
// blocks, 3 panels of 512 columns) left most of the chip idle and made each
// block's whole entry list one chain of dependent gathers.  V = 2 (4 columns
// a lane, 8-byte gathers) halves the minima's registers and the LDS the
// partial minima pass through, so more workgroups fit a CU and U can grow.
//
// With `info` set, the items are the parts of the row blocks instead of the
// blocks (entries ptr[f] .. ptr[f+1]-1 of part f, info[f] = block << 16 | the
// part's row mask): a part bound at half the longest block halves the
// longest run of entries a wave walks, for a few more gathers.
//
// T4: the tree stops at four waves, which all hand their minima to LDS; each
// then folds four of the 16 rows over the four and stores them (one round
// and two barriers fewer than halving down to wave 0, and four waves
// storing instead of one).
template <int U, int W, int V, int WPE, bool T4 = true>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE)))
block_split_step_kernel(
    int64_t N, int64_t nitems, const int64_t *__restrict__ bptr,
    const uint64_t *__restrict__ ent, const int32_t *__restrict__ border,
    const uint32_t *__restrict__ info, const uint16_t *__restrict__ X, int64_t ldx,
    uint16_t *__restrict__ Y, int64_t ldy, int64_t ncols) {
  typedef typename ChunkOf<V>::type chunk;
  static_assert(!T4 || W >= 4, "four waves at least");
  constexpr int kSlots = (T4 && W / 2 < 4) ? 4 : W / 2;
  __shared__ uint32_t part[kSlots][kRows * V][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / nitems;
  const int64_t bslot = t - panel * nitems;
  const int64_t it = border ? (int64_t)((kconst_i32)border)[bslot] : bslot;
  uint32_t rows = 0xFFFFu;
  int64_t b = it;
  if (info) {
    const uint32_t w = ((kconst_u32)info)[it];
    b = w >> 16;
    rows = w & 0xFFFFu;
  }
  const int64_t c0 = (panel * 64 + lane) * (2 * V);
  const kconst_i64 bp = (kconst_i64)bptr;
  const kconst_u64 en = (kconst_u64)ent;
  const gconst<chunk> Xg = (gconst<chunk>)to_global(X);
  const int64_t ldc = ldx / (2 * V);
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / (2 * V)) : 0u;

  u16x2 acc[kRows][V];
#pragma unroll
  for (int r = 0; r < kRows; ++r)
#pragma unroll
    for (int k = 0; k < V; ++k) acc[r][k] = splat(0xFFFFu);
  const int64_t e0 = bp[it], e1 = bp[it + 1];
  const int64_t per = (e1 - e0 + W - 1) / W;
  const int64_t my0 = e0 + (int64_t)wave * per, my1 = min(e1, my0 + per);
  block_entries<U, V>(en, my0, my1, Xg, ldc, off, acc);
  // the W partial minima meet in LDS, halving the waves each round
#pragma unroll 1
  for (int half = W / 2; half >= (T4 ? 4 : 1); half /= 2) {
    if (wave >= half && wave < 2 * half) {
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < V; ++k) part[wave - half][r * V + k][lane] = as_u32(acc[r][k]);
    }
    __syncthreads();
    if (wave < half) {
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < V; ++k)
          acc[r][k] = pk_min(acc[r][k], as_pk(part[wave][r * V + k][lane]));
    }
    __syncthreads();
  }
  if constexpr (T4) {
    if (wave < 4) {
#pragma unroll
      for (int r = 0; r < kRows; ++r)
#pragma unroll
        for (int k = 0; k < V; ++k) part[wave][r * V + k][lane] = as_u32(acc[r][k]);
    }
    __syncthreads();
    if (wave >= 4 || c0 >= ncols) return;
#pragma unroll
    for (int i = 0; i < kRows / 4; ++i) {
      const int r = wave * (kRows / 4) + i;
      const int64_t q = b * kRows + r;
      if (q >= N || !(rows & (1u << r))) continue;
      u16x2 m[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        m[k] = as_pk(part[0][r * V + k][lane]);
#pragma unroll
        for (int w = 1; w < 4; ++w) m[k] = pk_min(m[k], as_pk(part[w][r * V + k][lane]));
      }
      if (c0 + 2 * V <= ncols) {
        chunk o;
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = as_u32(m[k]);
        *(gmut<chunk>)(to_global_mut(Y) + q * ldy + c0) = o;
      } else {
        const gmut<uint16_t> y = to_global_mut(Y) + q * ldy + c0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
          if (c0 + 2 * k < ncols) y[2 * k] = m[k].x;
          if (c0 + 2 * k + 1 < ncols) y[2 * k + 1] = m[k].y;
        }
      }
    }
    return;
  }
  if (wave != 0 || c0 >= ncols) return;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int64_t q = b * kRows + r;
    if (q >= N) break;
    if (!(rows & (1u << r))) continue;
    const u16x2 *a = acc[r];
    if (c0 + 2 * V <= ncols) {
      chunk o;
#pragma unroll
      for (int k = 0; k < V; ++k) o[k] = as_u32(a[k]);
      *(gmut<chunk>)(to_global_mut(Y) + q * ldy + c0) = o;
    } else {
      const gmut<uint16_t> y = to_global_mut(Y) + q * ldy + c0;
#pragma unroll
      for (int k = 0; k < V; ++k) {
        if (c0 + 2 * k < ncols) y[2 * k] = a[k].x;
        if (c0 + 2 * k + 1 < ncols) y[2 * k + 1] = a[k].y;
      }
    }
  }
}

// The grouped step on row-block parts (small n): one (part, 256-column
// panel) item per workgroup of four waves (part_rows), parts by decreasing
// entry count, each XCD a contiguous range of items.  The parts cap the
// entries any wave walks at a quarter of the part bound, the 16 rows' minima
// of 4 columns a lane take 32 registers, and only four partial minima meet
// in 16 KB of LDS, so a CU holds eight such workgroups: at n = 8 every item
// is resident at once, where the workgroup-shared blocks (16 waves, 128 KB
// of LDS, one workgroup per CU) needed two rounds and spent half their time
// combining the 16 partial minima.
template <int U>
__global__ void __launch_bounds__(256) part_step_kernel(
    int64_t N, int64_t nf, const int64_t *__restrict__ fptr, const uint64_t *__restrict__ fent,
    const uint32_t *__restrict__ finfo, const int32_t *__restrict__ forder,
    const uint16_t *__restrict__ X, int64_t ldx, uint16_t *__restrict__ Y, int64_t ldy,
    int64_t ncols) {
  __shared__ uint32_t part[4 * kRows * 2 * 64];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t panel = t / nf;
  const int64_t f = ((kconst_i32)forder)[t - panel * nf];
  part_rows<U, 2, 4>((kconst_i64)fptr, (kconst_u64)fent, (kconst_u32)finfo, f, X, ldx, Y, ldy,
                     N, ncols, panel * 256 + (int64_t)lane * 4, wv, lane,
                     (__attribute__((address_space(3))) uint32_t *)part);
}

hipError_t launch_block_step_u16(int64_t N, const int64_t *bptr, const uint64_t *ent,
                                 const int32_t *border, const FineView *fine, const uint16_t *X,
                                 int64_t ldx, uint16_t *Y, int64_t ldy, int64_t ncols,
                                 bool grouped, hipStream_t s) {
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
  // the chip (n >= 10); below that a workgroup of 8 waves shares each block
  // (n = 9) or part of a block (n = 8); up to n = 7 four waves take each
  // part at 4 columns a lane
  const int64_t items = nblocks * panels;
  const bool pipe_ok = vec && ldx >= (ncols + 7) / 8 * 8;
  // parts: 8-byte chunks of rows at least ncols rounded up to 4 long
  const bool parts_ok = fine && fine->nf > 0 && (ldx % 4 == 0) && (ldy % 4 == 0) &&
                        ((uintptr_t)X % 8 == 0) && ((uintptr_t)Y % 8 == 0) &&
                        ldx >= (ncols + 3) / 4 * 4;
  if (parts_ok && grouped && N <= 1024) {
    const int64_t pitems = fine->nf * ((ncols + 255) / 256);
    hipLaunchKernelGGL(part_step_kernel<4>, dim3((unsigned)pitems), dim3(256), 0, s, N, fine->nf,
                       fine->fptr, fine->fent, fine->finfo, fine->forder, X, ldx, Y, ldy, ncols);
  } else if (pipe_ok && grouped && parts_ok && N <= 2048) {
    // n = 8: the parts (17.6 us against 18.5 on the blocks, 20.4 with 16
    // waves a block)
    const int64_t pitems = fine->nf * panels;
    hipLaunchKernelGGL((block_split_step_kernel<4, 8, 4, 4>), dim3((unsigned)pitems), dim3(512),
                       0, s, N, fine->nf, fine->fptr, fine->fent, fine->forder, fine->finfo, X,
                       ldx, Y, ldy, ncols);
  } else if (pipe_ok && grouped && items < 4096)
    hipLaunchKernelGGL((block_split_step_kernel<4, 8, 4, 4>), dim3((unsigned)items), dim3(512), 0,
                       s, N, nblocks, bptr, ent, border, nullptr, X, ldx, Y, ldy, ncols);
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
                             const int32_t *border, const FineView *fine, const uint16_t *X,
                             int64_t ldx, uint16_t *Y, int64_t ldy, int64_t ncols, bool grouped,
                             hipStream_t s) {
  if (N == 0 || ncols == 0) return hipSuccess;
  return launch_block_step_u16(N, bptr, ent, border, fine, X, ldx, Y, ldy, ncols, grouped, s);
}

}  // namespace tp
