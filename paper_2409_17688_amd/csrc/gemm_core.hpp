// The (min,+) product of one BM x BN tile of C, shared by the one-shot
// product kernel and the persistent batch kernel (Section 1:
// (A x B)_ij = min_k a_ik + b_kj).
//
// Design for gfx950.  (min,+) has no multiply, so matrix cores do not apply;
// the product runs on the vector ALUs with two 16-bit lanes per 32-bit
// register: one v_pk_add_u16 with clamp (saturating, so INF = 65535 absorbs)
// and one v_pk_min_u16 per two (min,+) operations.  That makes the ceiling
// one (min,+) operation per lane per clock.
//   * 256 lanes (4 waves) own the tile; each lane owns TM x TN outputs held
//     as TM * TN / 2 packed registers.
//   * K advances in slabs of BK.  The A slab is stored k-major in LDS (so the
//     TM values a lane needs at one k are one 16-byte read) and the B slab
//     row-major; both are double-buffered, and the next slab's global loads
//     are issued before the current slab's arithmetic, so one barrier per
//     slab suffices.
//   * The a_ik value is broadcast into both halves by the instruction's
//     op_sel bits, so the inner loop is nothing but packed add/min pairs and
//     a few LDS reads.
//   * 8-bit storage (INF = 255) is widened to 16 bits on the way into LDS;
//     results are clamped to 255 on the way out, which is exact because
//     min_k min(a + b, 255) = min(min_k (a + b), 255).
//   * Ragged edges are filled with the storage INF in LDS, which never wins a
//     min.
#pragma once

#include "common.hpp"

namespace tp {

template <typename T>
struct Storage;
template <>
struct Storage<uint16_t> {
  static constexpr uint16_t inf = 0xFFFFu;
};
template <>
struct Storage<uint8_t> {
  static constexpr uint16_t inf = 0xFFu;
};

constexpr int kGemmThreads = 256;

// One 16-byte chunk of a row: VE consecutive elements starting at (row, col).
// Elements outside [0, rows) x [0, cols) read as the storage INF.
template <typename T, bool VEC>
__device__ __forceinline__ uint4 load_chunk(const T *__restrict__ base, int64_t ld, int row,
                                            int col, int rows, int cols) {
  constexpr int VE = 16 / sizeof(T);
  const gconst<T> p = to_global(base) + (int64_t)row * ld + col;
  if (VEC && row < rows && col + VE <= cols) return gload16<T>(p);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < VE; ++e) {
    const uint32_t v = (row < rows && col + e < cols) ? (uint32_t)p[e] : (uint32_t)Storage<T>::inf;
    w[e / (VE / 4)] |= v << ((e % (VE / 4)) * 8 * sizeof(T));
  }
  return uint4{w[0], w[1], w[2], w[3]};
}

// Element e (0..VE-1) of a chunk, widened to 16 bits.
template <typename T>
__device__ __forceinline__ uint16_t chunk_elem(const uint4 &c, int e) {
  const uint32_t w[4] = {c.x, c.y, c.z, c.w};
  if constexpr (sizeof(T) == 2)
    return (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
  else
    return (uint16_t)((w[e >> 2] >> (8 * (e & 3))) & 0xFFu);
}

// C[m0 .. m0+BM) x [n0 .. n0+BN) = A x B (accumulate != 0: min with the old C).
// All 256 lanes of the workgroup call it; As and Bs are LDS buffers of
// 2 x BK x BM and 2 x BK x BN entries.  Ends with the epilogue stores (no
// trailing barrier: the caller synchronizes before reusing the buffers).
// u8 entries are summed in 16 bits and stored clamped to 255.  For u8
// operands that are residuals over a base (255 out of range, not INF):
// `sub` is subtracted from every sum before the clamp, a tile that clamps an
// entry sets bit 1 of *sat, and each wave folds the least entry it stores
// into *least (atomic min).
template <int BM, int BN, int BK, int TM, int TN, typename T, bool VEC>
__device__ __forceinline__ void gemm_tile(int M, int N, int K, const T *__restrict__ A,
                                          int64_t lda, const T *__restrict__ B, int64_t ldb,
                                          T *__restrict__ C, int64_t ldc, int accumulate, int m0,
                                          int n0, uint16_t (*As)[BK][BM], uint16_t (*Bs)[BK][BN],
                                          int32_t *sat = nullptr, uint16_t sub = 0,
                                          int32_t *least = nullptr) {
  constexpr int kThreads = kGemmThreads;
  static_assert((BM / TM) * (BN / TN) == kThreads, "thread layout");
  static_assert(TM % 8 == 0 || TM == 4, "A fragment");
  static_assert(TN % 8 == 0 || TN == 4, "B fragment");
  constexpr int VE = 16 / sizeof(T);  // elements per 16-byte global load
  constexpr int A_TOTAL = BM * BK / VE, B_TOTAL = BK * BN / VE;  // 16-byte chunks per slab
  constexpr int A_VECS = (A_TOTAL + kThreads - 1) / kThreads;
  constexpr int B_VECS = (B_TOTAL + kThreads - 1) / kThreads;
  static_assert(A_TOTAL % kThreads == 0 || A_TOTAL < kThreads, "A slab split");
  static_assert(B_TOTAL % kThreads == 0 || B_TOTAL < kThreads, "B slab split");
  constexpr int TM2 = TM / 2, TN2 = TN / 2;

  const int tid = threadIdx.x;
  const int tm = tid / (BN / TN), tn = tid % (BN / TN);

  uint4 ra[A_VECS], rb[B_VECS];

  auto global_load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < A_VECS; ++i) {
      const int v = tid + i * kThreads;
      if (A_TOTAL < kThreads && v >= A_TOTAL) break;
      const int row = v / (BK / VE), kv = v % (BK / VE);
      ra[i] = load_chunk<T, VEC>(A, lda, m0 + row, k0 + kv * VE, M, K);
    }
#pragma unroll
    for (int i = 0; i < B_VECS; ++i) {
      const int v = tid + i * kThreads;
      if (B_TOTAL < kThreads && v >= B_TOTAL) break;
      const int krow = v / (BN / VE), nv = v % (BN / VE);
      rb[i] = load_chunk<T, VEC>(B, ldb, k0 + krow, n0 + nv * VE, K, N);
    }
  };
  auto lds_store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_VECS; ++i) {
      const int v = tid + i * kThreads;
      if (A_TOTAL < kThreads && v >= A_TOTAL) break;
      const int row = v / (BK / VE), kv = v % (BK / VE);
#pragma unroll
      for (int e = 0; e < VE; ++e) As[buf][kv * VE + e][row] = chunk_elem<T>(ra[i], e);
    }
#pragma unroll
    for (int i = 0; i < B_VECS; ++i) {
      const int v = tid + i * kThreads;
      if (B_TOTAL < kThreads && v >= B_TOTAL) break;
      const int krow = v / (BN / VE), nv = v % (BN / VE);
      if constexpr (sizeof(T) == 2) {
        *reinterpret_cast<uint4 *>(&Bs[buf][krow][nv * VE]) = rb[i];
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          uint4 w;
          w.x = chunk_elem<T>(rb[i], 8 * h + 0) | ((uint32_t)chunk_elem<T>(rb[i], 8 * h + 1) << 16);
          w.y = chunk_elem<T>(rb[i], 8 * h + 2) | ((uint32_t)chunk_elem<T>(rb[i], 8 * h + 3) << 16);
          w.z = chunk_elem<T>(rb[i], 8 * h + 4) | ((uint32_t)chunk_elem<T>(rb[i], 8 * h + 5) << 16);
          w.w = chunk_elem<T>(rb[i], 8 * h + 6) | ((uint32_t)chunk_elem<T>(rb[i], 8 * h + 7) << 16);
          *reinterpret_cast<uint4 *>(&Bs[buf][krow][nv * VE + 8 * h]) = w;
        }
      }
    }
  };
  // The TM values of A and TN values of B one lane needs at step k.
  auto lds_frag = [&](int buf, int k, u16x2 (&a2)[TM2], u16x2 (&b2)[TN2]) {
    if constexpr (TM % 8 == 0) {
#pragma unroll
      for (int v = 0; v < TM / 8; ++v) {
        const uint4 w = *reinterpret_cast<const uint4 *>(&As[buf][k][tm * TM + v * 8]);
        a2[4 * v + 0] = as_pk(w.x);
        a2[4 * v + 1] = as_pk(w.y);
        a2[4 * v + 2] = as_pk(w.z);
        a2[4 * v + 3] = as_pk(w.w);
      }
    } else {
      const uint2 w = *reinterpret_cast<const uint2 *>(&As[buf][k][tm * TM]);
      a2[0] = as_pk(w.x);
      a2[1] = as_pk(w.y);
    }
    if constexpr (TN % 8 == 0) {
#pragma unroll
      for (int v = 0; v < TN / 8; ++v) {
        const uint4 w = *reinterpret_cast<const uint4 *>(&Bs[buf][k][tn * TN + v * 8]);
        b2[4 * v + 0] = as_pk(w.x);
        b2[4 * v + 1] = as_pk(w.y);
        b2[4 * v + 2] = as_pk(w.z);
        b2[4 * v + 3] = as_pk(w.w);
      }
    } else {
      const uint2 w = *reinterpret_cast<const uint2 *>(&Bs[buf][k][tn * TN]);
      b2[0] = as_pk(w.x);
      b2[1] = as_pk(w.y);
    }
  };

  u16x2 acc[TM][TN2];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN2; ++j) acc[i][j] = splat(0xFFFFu);

  const int nslab = (K + BK - 1) / BK;
  if (nslab > 0) {
    global_load(0);
    lds_store(0);
  }
  __syncthreads();

  // one step k of the slab: acc = min(acc, a_k + b_k) over the lane's tile
  auto step = [&](const u16x2 (&a2)[TM2], const u16x2 (&b2)[TN2]) {
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const u16x2 av = splat((i & 1) ? a2[i >> 1].y : a2[i >> 1].x);
      // all adds of the row first, then the mins: an add whose a_ik comes
      // from the high half (op_sel) followed at once by the min reading its
      // result costs a hazard wait state on gfx950; grouped, the results are
      // consumed TN/2 instructions later and no waits are inserted
      u16x2 sum[TN2];
#pragma unroll
      for (int j = 0; j < TN2; ++j) sum[j] = pk_add_sat(av, b2[j]);
#pragma unroll
      for (int j = 0; j < TN2; ++j) acc[i][j] = pk_min(acc[i][j], sum[j]);
    }
  };
  static_assert(BK % 2 == 0, "the slab is walked two steps at a time");

  for (int s = 0; s < nslab; ++s) {
    const int buf = s & 1;
    if (s + 1 < nslab) global_load((s + 1) * BK);
    // two fragment sets in turn: the fragments of the next step are
    // requested before the arithmetic of the current one, and no registers
    // are copied from one step to the next
    u16x2 a0[TM2], b0[TN2], a1[TM2], b1[TN2];
    lds_frag(buf, 0, a0, b0);
#pragma unroll 1
    for (int k = 0; k < BK - 2; k += 2) {
      lds_frag(buf, k + 1, a1, b1);
      step(a0, b0);
      lds_frag(buf, k + 2, a0, b0);
      step(a1, b1);
    }
    lds_frag(buf, BK - 1, a1, b1);
    step(a0, b0);
    step(a1, b1);
    if (s + 1 < nslab) lds_store(buf ^ 1);
    __syncthreads();
  }

  // epilogue
  constexpr uint16_t OUT_INF = Storage<T>::inf;
  bool clamped = false;
  int32_t low = 0xFFFF;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int r = m0 + tm * TM + i;
    if (r >= M) continue;
    const gmut<T> crow = to_global_mut(C) + (int64_t)r * ldc;
#pragma unroll
    for (int j = 0; j < TN2; ++j) {
      const int c = n0 + tn * TN + 2 * j;
      u16x2 v = acc[i][j];
      if constexpr (sizeof(T) == 1) {
        if (sat) {
          v = __builtin_elementwise_sub_sat(v, splat(sub));
          clamped |= (c < N && v.x >= OUT_INF) || (c + 1 < N && v.y >= OUT_INF);
          if (c < N) low = min(low, (int32_t)v.x);
          if (c + 1 < N) low = min(low, (int32_t)v.y);
        }
        v = pk_min(v, splat(OUT_INF));
      }
      if (c + 1 < N) {
        if (accumulate) {
          const u16x2 old = u16x2{(uint16_t)crow[c], (uint16_t)crow[c + 1]};
          v = pk_min(v, old);
        }
        if constexpr (sizeof(T) == 2) {
          if (VEC)
            *(gmut<uint32_t>)(crow + c) = as_u32(v);
          else {
            crow[c] = v.x;
            crow[c + 1] = v.y;
          }
        } else {
          crow[c] = (T)v.x;
          crow[c + 1] = (T)v.y;
        }
      } else if (c < N) {
        uint16_t x = v.x;
        if (accumulate) x = min(x, (uint16_t)crow[c]);
        crow[c] = (T)x;
      }
    }
  }
  if (sat && clamped) atomicOr(sat, 1);
  if (least) {
    for (int off = 32; off > 0; off >>= 1) low = min(low, __shfl_xor(low, off));
    if ((threadIdx.x & 63) == 0 && low < 0xFFFF) atomicMin(least, low);
  }
}


}  // namespace tp
