// Device building blocks shared by the one-shot kernels and the persistent
// batch kernel: the "can follow" test, one 16-byte chunk of a sparse left
// product row, and one 64 x 64 tile of a trace of a product.
#pragma once

#include "common.hpp"

namespace tp {

// p can follow q (Section 2.2).  Masks hold the zeros of a word in bits
// 0..15 and its ones in bits 16..31; `full` has the low n bits set.  With
// x = zeros of q, y = zeros of p shifted to the next position, w = zeros of p
// shifted to the previous one, "exactly one zero among q_i, p_{i-1}, p_{i+1}"
// and "at least two" are bitwise functions of x, y, w.
__device__ __forceinline__ bool can_follow(uint32_t mq, uint32_t mp, uint32_t full) {
  const uint32_t zq = mq & 0xFFFFu, oq = mq >> 16, tq = full & ~(zq | oq);
  const uint32_t zp = mp & 0xFFFFu, op = mp >> 16, tp = full & ~(zp | op);
  const uint32_t x = zq, y = (zp << 1) & full, w = zp >> 1;
  const uint32_t exactly_one = (x ^ y ^ w) & ~(x & y & w);
  const uint32_t two_or_more = (x & y) | (x & w) | (y & w);
  return ((tq & ~zp) | (tp & ~exactly_one) | (op & ~two_or_more)) == 0;
}

template <typename T>
__device__ __forceinline__ uint16_t storage_inf() {
  return sizeof(T) == 2 ? (uint16_t)0xFFFFu : (uint16_t)0xFFu;
}

// 16 bytes of row `row` of X from column `col`, as packed 16-bit pairs;
// columns >= ncols read as the storage INF.
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
      const uint16_t x0 = c0 < ncols ? (uint16_t)p[2 * e] : storage_inf<T>();
      const uint16_t x1 = c1 < ncols ? (uint16_t)p[2 * e + 1] : storage_inf<T>();
      out[e] = u16x2{x0, x1};
    }
  }
}

// Y[q][c0 .. c0+VE) = min over successors p of q of (z_p + X[p][c0 ..]):
// one lane's chunk of row q of the sparse left product.  The successor list
// is the same for every lane of the wave; U successor rows are in flight per
// lane.
template <typename T, bool VEC, int U = 8>
__device__ __forceinline__ void spmm_row_chunk(const int64_t *__restrict__ rowptr,
                                               const uint32_t *__restrict__ col,
                                               const uint8_t *__restrict__ z,
                                               const T *__restrict__ X, int64_t ldx,
                                               T *__restrict__ Y, int64_t ldy, int64_t ncols,
                                               int64_t q, int64_t c0) {
  constexpr int VE = 16 / sizeof(T);
  constexpr int P = VE / 2;  // packed registers per lane
  const int64_t begin = rowptr[q], end = rowptr[q + 1];
  u16x2 acc[P];
#pragma unroll
  for (int e = 0; e < P; ++e) acc[e] = splat(0xFFFFu);
  int64_t e = begin;
  for (; e + U <= end; e += U) {
    u16x2 v[U][P];
    uint16_t lab[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = col[e + u];
      lab[u] = z[p];
      load_row_chunk<T, VEC>(X, ldx, p, c0, ncols, v[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
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

// Row q (wave-uniform) of Y = A(D_n) x X over this lane's 8 columns
// c0 .. c0 + 7 (u16; ldx, ldy and c0 multiples of 8, X 16-byte aligned, X's
// rows at least ncols rounded up to 8 long, so the 8 entries exist even past
// ncols; only columns < ncols are stored), from the
// packed successor list colz (successor in bits 0..23, its label z_p in bits
// 24..31), read with scalar loads.  Software-pipelined: the next U
// successors' indices and rows are requested before the current U are
// combined, so two rounds of gathers are in flight.  A last partial round
// repeats the row's last successor with an INF label, which never wins.
template <int U>
__device__ __forceinline__ void gather_row_colz(kconst_i64 rowptr, kconst_u32 colz,
                                                const uint16_t *X, int64_t ldx, uint16_t *Y,
                                                int64_t ldy, int64_t ncols, int64_t q,
                                                int64_t c0) {
  const int64_t b = rowptr[q], e = rowptr[q + 1];
  const gconst<u32x4> Xg = (gconst<u32x4>)to_global(X);
  const int64_t ld4 = ldx / 8;
  // lanes past the last column read chunk 0 of each row (inside the row) and
  // store nothing
  const uint32_t off = c0 < ncols ? (uint32_t)(c0 / 8) : 0u;
  u16x2 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = splat(0xFFFFu);
  if (b < e) {
    const int64_t last = e - 1;
    auto fetch = [&](int64_t i, uint32_t (&pz)[U], u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = i + u;
        const uint32_t w = colz[k < last ? k : last];
        pz[u] = k <= last ? w : (w | 0xFF000000u);
        v[u] = Xg[(int64_t)(pz[u] & 0xFFFFFFu) * ld4 + off];
      }
    };
    auto combine = [&](const uint32_t (&pz)[U], const u32x4 (&v)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t z = pz[u] >> 24;
        const u16x2 lab = splat((uint16_t)(z == 0xFFu ? 0xFFFFu : z));
        acc[0] = pk_min(acc[0], pk_add_sat(lab, as_pk(v[u].x)));
        acc[1] = pk_min(acc[1], pk_add_sat(lab, as_pk(v[u].y)));
        acc[2] = pk_min(acc[2], pk_add_sat(lab, as_pk(v[u].z)));
        acc[3] = pk_min(acc[3], pk_add_sat(lab, as_pk(v[u].w)));
      }
    };
    uint32_t pa[U], pb[U];
    u32x4 va[U], vb[U];
    fetch(b, pa, va);
    for (int64_t i = b;;) {
      bool more = i + U <= last;
      if (more) fetch(i + U, pb, vb);
      combine(pa, va);
      i += U;
      if (!more) break;
      more = i + U <= last;
      if (more) fetch(i + U, pa, va);
      combine(pb, vb);
      i += U;
      if (!more) break;
    }
  }
  if (c0 >= ncols) return;
  if (c0 + 8 <= ncols) {
    *(gmut<u32x4>)(to_global_mut(Y) + q * ldy + c0) =
        u32x4{as_u32(acc[0]), as_u32(acc[1]), as_u32(acc[2]), as_u32(acc[3])};
  } else {
    const gmut<uint16_t> y = to_global_mut(Y) + q * ldy + c0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (c0 + 2 * r < ncols) y[2 * r] = acc[r].x;
      if (c0 + 2 * r + 1 < ncols) y[2 * r + 1] = acc[r].y;
    }
  }
}

// Rows per block of the blocked form of A(D_n).
constexpr int kBlockRows = 16;

// acc[r] = min(acc[r], g) for the rows r whose bit is set in m.
template <int V>
__device__ __forceinline__ void apply_group(u16x2 (&acc)[kBlockRows][V], uint32_t m,
                                            const u16x2 (&g)[V]) {
#pragma unroll
  for (int r = 0; r < kBlockRows; ++r) {
    if (m & (1u << r)) {
#pragma unroll
      for (int k = 0; k < V; ++k) acc[r][k] = pk_min(acc[r][k], g[k]);
    }
  }
}

// Entries [i0, i1) of a block's entry list (grouped by row mask, bit 48 on
// the last entry of each group; entry layout: successor p in bits 0..23, its
// label z_p in 24..31, row mask in 32..47) folded into acc, the block's rows
// at this lane's 2V columns: each entry gathers 4V bytes of row p of X (chunk
// `off` of the row, ldc chunks per row), adds z_p and takes the minimum into
// its group's running minimum, which goes to the rows of the group's mask at
// the group's end.  The range may start or end inside a group: its last
// entry closes the group it is in, so every partial group still reaches its
// rows.  Two rounds of U gathers are in flight; the entries are uniform in
// the wave and read with scalar loads, a round ahead of their gathers.
template <int V> struct ChunkOf;
template <> struct ChunkOf<2> { typedef u32x2 type; };
template <> struct ChunkOf<4> { typedef u32x4 type; };

template <int U, int V = 4>
__device__ __forceinline__ void block_entries(kconst_u64 en, int64_t i0, int64_t i1,
                                              gconst<typename ChunkOf<V>::type> Xg, int64_t ldc,
                                              uint32_t off, u16x2 (&acc)[kBlockRows][V]) {
  typedef typename ChunkOf<V>::type chunk;
  if (i0 >= i1) return;
  u16x2 g[V];
#pragma unroll
  for (int k = 0; k < V; ++k) g[k] = splat(0xFFFFu);
  // entry indices in 32 bits (a state matrix's blocked form has far fewer
  // than 2^32 entries), so the range tests and clamps are single scalar ops
  const uint32_t first = (uint32_t)i0, last = (uint32_t)(i1 - 1);
  // the entries of the next round are loaded a round ahead (scalar loads
  // return out of order, so a gather right after its entry's load would wait
  // for every scalar load in flight); a round inside the range is one
  // scalar load of U consecutive entries
  uint64_t nx[U];
  typedef uint64_t round_t __attribute__((ext_vector_type(U), aligned(8)));
  auto load_entries = [&](uint32_t i) {
    if (i + (U - 1) <= last) {
      const round_t r = *(const __attribute__((address_space(4))) round_t *)(en + i);
#pragma unroll
      for (int u = 0; u < U; ++u) nx[u] = r[u];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) nx[u] = en[min(i + u, last)];
    }
  };
  auto fetch = [&](uint32_t i, uint64_t (&w)[U], chunk (&v)[U]) {
    if (i + (U - 1) < last) {
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = nx[u];
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t k = i + u;
        const uint64_t x = nx[u];
        // the range's last entry closes its group; past it: no rows, no
        // group end
        w[u] = k < last ? x : (k == last ? (x | kGroupEnd) : (x & 0xFFFFFFFFull));
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = Xg[(int64_t)(uint32_t)(nx[u] & 0xFFFFFFu) * ldc + off];
    load_entries(i + U);
  };
  auto apply = [&](const uint64_t (&w)[U], const chunk (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const u16x2 lab = splat((uint16_t)((w[u] >> 24) & 0xFFu));
#pragma unroll
      for (int k = 0; k < V; ++k) g[k] = pk_min(g[k], pk_add_sat(lab, as_pk(v[u][k])));
      if (w[u] & kGroupEnd) {
        apply_group<V>(acc, (uint32_t)(w[u] >> 32) & 0xFFFFu, g);
#pragma unroll
        for (int k = 0; k < V; ++k) g[k] = splat(0xFFFFu);
      }
    }
  };
  uint64_t wa[U], wb[U];
  chunk va[U], vb[U];
  load_entries(first);
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

// One (part f, 128V-column panel) item of Y = A x X on row-block parts, for
// a workgroup of four waves: each wave folds a quarter of the part's
// entries into the 16 rows' minima at its lane's 2V columns (16V
// registers).  The minima meet in `part`, S slots of LDS ([S][16 rows x
// V][64] words, 4 S V KB): with S = 2 waves 2 and 3 first hand theirs to
// waves 0 and 1; then the S waves write theirs and each folds 16 / S of the
// rows over the S slots and stores those of the part's mask (S waves
// storing, not one).  Columns c0 .. c0+2V-1 of X and Y, c0 < ncols for the
// lanes that store; X rows are whole 4V-byte chunks (ldx % 2V == 0).  Every
// wave of the workgroup must call it with the same item.
template <int U, int V, int S>
__device__ __forceinline__ void part_rows(kconst_i64 fptr, kconst_u64 fent, kconst_u32 finfo,
                                          int64_t f, const uint16_t *X, int64_t ldx, uint16_t *Y,
                                          int64_t ldy, int64_t N, int64_t ncols, int64_t c0,
                                          int wv, int lane,
                                          __attribute__((address_space(3))) uint32_t *part) {
  typedef typename ChunkOf<V>::type chunk;
  const uint32_t info = finfo[f];
  const int64_t b = info >> 16;
  const uint32_t rows = info & 0xFFFFu;
  const int64_t e0 = fptr[f], e1 = fptr[f + 1];
  const int64_t per = (e1 - e0 + 3) / 4;
  const int64_t my0 = e0 + (int64_t)wv * per, my1 = min(e1, my0 + per);
  u16x2 acc[kBlockRows][V];
#pragma unroll
  for (int r = 0; r < kBlockRows; ++r)
#pragma unroll
    for (int k = 0; k < V; ++k) acc[r][k] = splat(0xFFFFu);
  block_entries<U, V>(fent, my0, my1, (gconst<chunk>)to_global(X), ldx / (2 * V),
                      c0 < ncols ? (uint32_t)(c0 / (2 * V)) : 0u, acc);
  static_assert(S == 2 || S == 4, "two or four slots");
  if constexpr (S == 2) {
    if (wv >= 2) {
#pragma unroll
      for (int r = 0; r < kBlockRows; ++r)
#pragma unroll
        for (int k = 0; k < V; ++k)
          part[((wv - 2) * kBlockRows * V + r * V + k) * 64 + lane] = as_u32(acc[r][k]);
    }
    __syncthreads();
    if (wv < 2) {
#pragma unroll
      for (int r = 0; r < kBlockRows; ++r)
#pragma unroll
        for (int k = 0; k < V; ++k)
          acc[r][k] = pk_min(acc[r][k], as_pk(part[(wv * kBlockRows * V + r * V + k) * 64 + lane]));
    }
    __syncthreads();
  }
  if (wv < S) {
#pragma unroll
    for (int r = 0; r < kBlockRows; ++r)
#pragma unroll
      for (int k = 0; k < V; ++k)
        part[(wv * kBlockRows * V + r * V + k) * 64 + lane] = as_u32(acc[r][k]);
  }
  __syncthreads();
  if (wv < S && c0 < ncols) {
#pragma unroll
    for (int i = 0; i < kBlockRows / S; ++i) {
      const int r = wv * (kBlockRows / S) + i;
      const int64_t q = b * kBlockRows + r;
      if (!(rows & (1u << r)) || q >= N) continue;
      u16x2 m[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        m[k] = as_pk(part[(r * V + k) * 64 + lane]);
#pragma unroll
        for (int w = 1; w < S; ++w)
          m[k] = pk_min(m[k], as_pk(part[(w * kBlockRows * V + r * V + k) * 64 + lane]));
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
  }
  // the slots are read before the workgroup's next item writes them
  __syncthreads();
}

// Eight consecutive entries of row `row` from column `col`, widened to 16
// bits; entries outside [0, n) x [0, n) read as 0xFFFF.
template <typename T, bool VEC>
__device__ __forceinline__ uint4 load8(const T *__restrict__ M, int64_t ld, int64_t row,
                                       int64_t col, int64_t n) {
  const gconst<T> p = to_global(M) + row * ld + col;
  if (VEC && row < n && col + 8 <= n) {
    if constexpr (sizeof(T) == 2) {
      return gload16<T>(p);
    } else {
      const uint2 v = gload8<T>(p);
      return uint4{__builtin_amdgcn_perm(0u, v.x, 0x0c010c00u),
                   __builtin_amdgcn_perm(0u, v.x, 0x0c030c02u),
                   __builtin_amdgcn_perm(0u, v.y, 0x0c010c00u),
                   __builtin_amdgcn_perm(0u, v.y, 0x0c030c02u)};
    }
  }
  uint32_t w[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t lo = (row < n && col + 2 * e < n) ? (uint32_t)p[2 * e] : 0xFFFFu;
    const uint32_t hi = (row < n && col + 2 * e + 1 < n) ? (uint32_t)p[2 * e + 1] : 0xFFFFu;
    w[e] = lo | (hi << 16);
  }
  return uint4{w[0], w[1], w[2], w[3]};
}

constexpr int kTraceLdsStride = 72;  // entries; 144-byte rows keep 16-byte reads aligned

// Folds min over i in [i0, i0+64), k in [k0, k0+64) of x_ik + y_ki into acc.
// Called by all 256 lanes of a workgroup; yt is 64 * kTraceLdsStride entries
// of LDS.  Ends with a barrier, so yt can be reused right away.
template <typename T, bool VEC>
__device__ __forceinline__ void trace_tile(const T *__restrict__ X, int64_t ldx,
                                           const T *__restrict__ Y, int64_t ldy, int64_t N,
                                           int64_t i0, int64_t k0, uint16_t *yt,
                                           u16x2 (&acc)[4]) {
  constexpr int S = kTraceLdsStride;
  const int tid = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = tid + h * 256;  // chunk: row kr of the Y tile, columns ch*8 .. ch*8+7
    const int kr = c >> 3, ch = c & 7;
    const uint4 v = load8<T, VEC>(Y, ldy, k0 + kr, i0 + ch * 8, N);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) yt[(ch * 8 + e) * S + kr] = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int c = tid + h * 256;  // chunk: row ir of the X tile, columns kc*8 .. kc*8+7
    const int ir = c >> 3, kc = c & 7;
    const uint4 xv = load8<T, VEC>(X, ldx, i0 + ir, k0 + kc * 8, N);
    const uint4 yv = *reinterpret_cast<const uint4 *>(&yt[ir * S + kc * 8]);
    acc[0] = pk_min(acc[0], pk_add_sat(as_pk(xv.x), as_pk(yv.x)));
    acc[1] = pk_min(acc[1], pk_add_sat(as_pk(xv.y), as_pk(yv.y)));
    acc[2] = pk_min(acc[2], pk_add_sat(as_pk(xv.z), as_pk(yv.z)));
    acc[3] = pk_min(acc[3], pk_add_sat(as_pk(xv.w), as_pk(yv.w)));
  }
  __syncthreads();
}

// Folds min over i in [i0, i0+64), k in [k0, k0+64) of x_ik + y_ki into acc,
// one wave per tile and no LDS: lane (kg, ig) = (lane / 8, lane % 8) reads the
// 8 x 8 blocks X[i0+8ig ..][k0+8kg ..] and Y[k0+8kg ..][i0+8ig ..] (per load,
// eight lanes cover 128 contiguous bytes of one row), transposes its Y block
// in registers (one byte permute per packed pair) and adds it to its X block.
// All 16 loads of a lane are in flight together.
template <typename T, bool VEC>
__device__ __forceinline__ void trace_tile_regs(const T *__restrict__ X, int64_t ldx,
                                                const T *__restrict__ Y, int64_t ldy, int64_t N,
                                                int64_t i0, int64_t k0, int lane,
                                                u16x2 (&acc)[4]) {
  const int ig = lane & 7, kg = lane >> 3;
  const int64_t i = i0 + 8 * ig, k = k0 + 8 * kg;
  uint4 xr[8], yr[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    xr[r] = load8<T, VEC>(X, ldx, i + r, k, N);
    yr[r] = load8<T, VEC>(Y, ldy, k + r, i, N);
  }
  auto word = [](const uint4 &v, int w) { return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w; };
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    // row i + r of X against column i + r of Y: y_{k+2c, i+r} and
    // y_{k+2c+1, i+r} packed like x_{i+r, k+2c} and x_{i+r, k+2c+1}
    const uint32_t sel = (r & 1) ? 0x07060302u : 0x05040100u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t yt = __builtin_amdgcn_perm(word(yr[2 * c + 1], r >> 1),
                                                word(yr[2 * c], r >> 1), sel);
      acc[c] = pk_min(acc[c], pk_add_sat(as_pk(word(xr[r], c)), as_pk(yt)));
    }
  }
}

// Minimum of the four packed accumulators over the whole workgroup (256
// lanes); the result is valid in lane 0.  `part` is 4 ints of LDS.
__device__ __forceinline__ int32_t block_min(const u16x2 (&acc)[4], int32_t *part) {
  const u16x2 m2 = pk_min(pk_min(acc[0], acc[1]), pk_min(acc[2], acc[3]));
  int32_t best = min((int32_t)m2.x, (int32_t)m2.y);
  for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
  __syncthreads();
  best = min(min(part[0], part[1]), min(part[2], part[3]));
  __syncthreads();
  return best;
}

}  // namespace tp
