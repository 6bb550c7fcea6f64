// Batched gamma_2: many (n, m) instances in one persistent launch.
//
// gamma_2(P_n x C_m) = min_i (A^m)_ii (Theorem 2) = the trace of A^a x A^b for
// any a + b = m, and the integer (min,+) semiring is associative, so any
// powers that add up to m give the same exact answer.  A context keeps, per
// path order n, a set of powers of A = A(D_n) resident in HBM:
//   babies  A^1 .. A^c      by the chain A^k = A x A^(k-1) of Algorithm 2,
//                           using the sparse left factor (nnz * N per level);
//   giants  A^(jc), j >= 2  by dense (min,+) products of two resident powers,
//                           j = h + (j - h) with h the largest power of two
//                           <= j (h = j/2 when j is a power of two itself),
//                           so J giants take about log2(J) rounds of
//                           independent products.
// Instance m is answered from two resident powers: m <= 2c by
// (ceil(m/2), floor(m/2)), otherwise m = jc + r with 1 <= r <= c by
// (jc, r).  Memory per n is (c + m_max/c) powers instead of m_max/2, and the
// number of sequential chain levels is c instead of m_max/2.
//
// A batch runs on the caller's stream in one of two modes:
//   split (default)  the chain levels A^1 .. A^c of every path order that
//      lacks them run first as plain launches of the library's sparse left
//      step, one stream per n (the steps of one n are sequential; different
//      n run side by side), then one persistent kernel runs the dense
//      products and the traces.  A chain level depends on the whole level
//      before it and fills the chip on its own, which a share of a
//      persistent kernel does not.
//   fused (TP_PARAM_FUSED_CHAIN)  everything, chain levels included, runs
//      in the one persistent launch: it first runs the chain level by level
//      (level k of every n that lacks A^k together), each level spread over
//      the whole grid, with a barrier over the grid between levels; then
//      the task list below.  A^1 is written from the masks, one (row,
//      512-column panel) item per wave; a level k >= 2 takes the row blocks
//      of A (16 rows, the union of their successors grouped by row mask, as
//      in the library's blocked step) cut by rows into parts of bounded
//      length, one (part, 512-column panel) item per workgroup, whose four
//      waves split the part's entries and meet in LDS; each XCD's
//      workgroups take the items of a range of columns, longest first, each
//      workgroup its next item from a counter when it is free.  The
//      barrier needs every workgroup resident at once, so this mode never
//      launches more workgroups than the chip holds, and such launches of
//      the process are ordered one after another on each device; a batch
//      that cannot get them all (the chip shared with other work that waits
//      too, such as another process's) ends at the wait limit like any other
//      stuck wait.
// The persistent kernel runs a list of tasks in dependency order:
//   GEMM   one 128 x 128 tile of A^(x+y) = A^x x A^y
//   TRACE  64 rows i of min_{i,k} (A^a)_ik + (A^b)_ki, folded into the
//          instance's result with an atomic min
// Dependencies are as narrow as the arithmetic allows, each a completion
// counter and a target count: a product tile (rows R, columns C) and a trace
// block (rows I) read rows R (I) of the left factor and columns C (I) of the
// right one, so a giant counts its finished tiles per 128-row and per
// 128-column block; chain powers are complete before the first task.
// The list is split into 8 queues, one per XCD, each keeping the list's
// order; a giant's tiles and an instance's trace blocks go to the queues in
// contiguous chunks.  Workgroups pop their own XCD's queue first (one atomic
// head per queue) and the others when it is empty.  Every dependency points
// to an earlier task of the list and a queue is only left when empty, so the
// earliest unfinished task is always held by a running workgroup and every
// wait ends; as a safety net each wait is bounded in time, and a timed-out
// wait sets an abort flag that makes every workgroup drain the queues
// without work.  A finished task publishes its rows with an agent-scope
// release (so the L2s of other XCDs see them) and counter increments; a
// workgroup acquires once per dependency it starts waiting on.  The kernel
// launch (counter reset, result reset, persistent kernel) is captured once
// in a hipGraph and replayed for every batch.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <vector>

#include "device_core.hpp"
#include "gemm_core.hpp"

namespace tp {

namespace {

enum : int32_t { kGemm = 2, kTrace = 3 };

struct Task {
  int32_t type, slot;
  int32_t out, x, y;           // exponents written / read
  int32_t row0, row1, c0, c1;  // rows and columns of the output block
  int32_t dep, dep_target;     // counters to wait for (-1: none) and the
  int32_t dep2, dep2_target;   //   counts they must reach
  int32_t done, done2;         // counters bumped when finished (-1: none)
  int32_t inst;                // instance of a TRACE
  int32_t queue;               // queue (XCD) the task is dealt to
  int32_t compact;             // operands (and output) are shared-base u8 powers
  int32_t done3;               // a compact giant's count of finished tiles (-1: none)
};

struct Slot {
  int32_t n, N;
  int64_t ld;
  uint32_t full;
  int32_t pad;
  const uint32_t *masks;
  const int64_t *rowptr;
  const uint32_t *colz;     // successors with their labels in the top byte
  uint16_t *const *powers;  // powers[e] = A^e for the exponents of this batch
  // shared-base compact powers (residuals u8, A^e = base[0] + residual)
  int64_t ld8;
  uint8_t *const *powers8;   // powers8[e]: residuals of A^e (or null)
  int32_t *const *bases8;    // bases8[e]: its base words
  // fused mode: row-block parts (entries fptr[f] .. fptr[f+1]-1 of fent,
  // finfo[f] = block << 16 | row mask)
  const int64_t *fptr;
  const uint64_t *fent;
  const uint32_t *finfo;
};

constexpr int kQueues = 8;  // one task queue per XCD

struct Control {
  int32_t head[kQueues];   // next task of each queue
  int32_t qbeg[kQueues];   // first task of each queue in the task array
  int32_t qcnt[kQueues];   // tasks in each queue
  int32_t abort;           // set when a wait exceeded the limit
  int32_t nlevels;         // fused mode: chain levels run before the tasks
  int64_t wait_limit;      // in s_memrealtime ticks (100 MHz)
  int32_t *status;         // bit 1: a compact product left its residual range
};

constexpr int kMaxSlots = 16;

// Fused mode: one chain level (exponent k) of every slot that needs it.  Its
// work items are (slot, panel, r) triples packed in 32 bits (slot in bits
// 28..31, panel in 20..27, r in 0..19), items[off .. off + count) of the
// launch's item list, all on 512-column panels.  Level 1 (A^1, from the
// masks): r is a row, one item per wave.  Levels k >= 2 (`parts` set): r is
// a part of a row block, one item per workgroup.  Their list is in column
// order (slot, then panel) cut into nx ranges of about equal work, xr[x] ..
// xr[x+1]-1, one for the workgroups of each XCD (workgroup g runs on XCD g
// mod 8, so each XCD gathers from a few column panels of A^(k-1)), each
// range by decreasing entry count.  The workgroups of XCD x take the items
// of its range in that order from a counter of their own, which only grows
// over the launch: every workgroup takes until it draws past the range, so
// a level moves the counter by the range's count plus its workgroups, and
// xbase[x] is where the level starts.  Levels of one kind with the same
// slots share one list.
constexpr int kXcds = 8;
struct Level {
  int32_t k, parts;
  int64_t off, count;
  int32_t nx;
  int32_t xr[kXcds + 1];
  int32_t xbase[kXcds];
};
__host__ __device__ constexpr uint32_t item_code(int slot, int64_t panel, int64_t q) {
  return ((uint32_t)slot << 28) | ((uint32_t)panel << 20) | (uint32_t)q;
}
// Level barrier counters at the start of the counter array, each on a
// 256-byte line of its own (atomics on one line serialize): workgroups per
// XCC, then the registrations, then arrivals per XCC and the XCCs done, the
// item counters of the XCDs, and the release of each XCC.  The arrival,
// done and release counters only grow: level L is complete at (L + 1) x the
// count.
constexpr int kLine = 64;  // int32 per line
constexpr int kMaxXcc = 16;
constexpr int kRegTotal = kMaxXcc, kArrive = kMaxXcc + 1, kXccDone = 2 * kMaxXcc + 1;
constexpr int kTake = 2 * kMaxXcc + 2;
constexpr int kRelease = kTake + kXcds;
constexpr int kLevelCounters = (kRelease + kMaxXcc) * kLine;
// XCC_ID hardware register (bits 3:0): which XCD, and so which L2, a wave is on
constexpr int kHwRegXccId = (3 << 11) | 20;
constexpr uint16_t kInf = 0xFFFFu;
constexpr int kPanel = 512;                       // columns of a chain level item: 64 lanes x 8
constexpr int kGBM = 128, kGBN = 128, kGBK = 32;  // dense product tile

__device__ __forceinline__ int32_t ld_relaxed(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until counters[dep] >= target.  Returns 0 when the batch
// was aborted (by this wait timing out or by another workgroup).  Task waits
// pause long between polls (hundreds of waiting workgroups polling one
// counter would otherwise crowd out the task pops and increments); barrier
// waits, which every workgroup enters at about the same time, poll often.
template <bool kBarrier = false>
__device__ __forceinline__ int wait_counter(const int32_t *counters, int dep, int target,
                                           Control *ctl, int64_t limit) {
  if (dep < 0) return 1;
  const uint64_t start = __builtin_amdgcn_s_memrealtime();
  while (ld_relaxed(&counters[dep]) < target) {
    if (ld_relaxed(&ctl->abort)) return 0;
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - start) > limit) {
      __hip_atomic_store(&ctl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0;
    }
    if (kBarrier)
      __builtin_amdgcn_s_sleep(4);  // ~256 clocks
    else
      __builtin_amdgcn_s_sleep(127);  // ~8000 clocks
  }
  return 1;
}

// Fused mode, chain level k >= 2: the workgroup's item (slot, 512-column
// panel, part of a row block) of A^k = A x A^(k-1) (part_rows: the four
// waves split the part's entries and meet in the LDS arena).  Slot fields
// are made wave-uniform so the entry loads are scalar loads.
__device__ __forceinline__ void part_item(const Slot *__restrict__ slots, uint32_t item, int lev,
                                          int wv, int lane, uint32_t *lds_words) {
  const uint32_t code = __builtin_amdgcn_readfirstlane(item);
  const Slot &sl = slots[code >> 28];
  const int64_t N = wave_uniform((int64_t)sl.N), ld = wave_uniform(sl.ld);
  const int64_t panel = (code >> 20) & 0xFFu, f = code & 0xFFFFFu;
  uint16_t *const *powers = wave_uniform(sl.powers);
  part_rows<4, 4, 2>((kconst_i64)wave_uniform(sl.fptr), (kconst_u64)wave_uniform(sl.fent),
                     (kconst_u32)wave_uniform(sl.finfo), f, wave_uniform(powers[lev - 1]), ld,
                     wave_uniform(powers[lev]), ld, N, N, panel * kPanel + (int64_t)lane * 8, wv,
                     lane, (__attribute__((address_space(3))) uint32_t *)lds_words);
}

__global__ void __launch_bounds__(256, 4) batch_kernel(Control *__restrict__ ctl,
                                                       const Task *__restrict__ tasks,
                                                       const Slot *__restrict__ slots,
                                                       const Level *__restrict__ levels,
                                                       const uint32_t *__restrict__ items,
                                                       int32_t *__restrict__ counters,
                                                       int32_t *__restrict__ results) {
  // one LDS arena: the dense product's A and B slabs, or a trace's Y tile
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * kGBK * kGBM + 2 * kGBK * kGBN];
  __shared__ int32_t part[4];
  __shared__ int32_t s_task, s_go;
  int acq_dep = -1, acq_dep2 = -1;  // dependencies this workgroup has acquired (thread 0)
  const int64_t limit = ctl->wait_limit;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the hardware deals workgroups to the XCDs in turn, so workgroup b runs on
  // XCD b mod 8 and serves that queue first; when it is empty it takes tasks
  // from the others, always in each queue's own order
  const int home = blockIdx.x % kQueues;

  // Fused mode: the chain levels first, level by level over all slots, every
  // workgroup taking a share of each level's (row, panel) items (one per
  // wave), with a barrier over the grid after each level.  Making a level's
  // rows visible to the other XCDs takes a write-back of the L2 holding
  // them; one per XCC and level is enough: every wave waits for its own
  // stores to reach its L2, the workgroup counts itself on its XCC's
  // arrival counter, and the last arrival of an XCC (the workgroups per XCC
  // are counted once at the start) writes that L2 back and counts the XCC.
  // That workgroup then waits (bounded) until all XCCs are in and releases
  // its XCC, whose other workgroups wait on that (a few pollers on the
  // global count instead of the whole grid), and every workgroup acquires.
  const int nlev = ctl->nlevels;
  if (nlev > 0) {
    __shared__ int32_t s_on_xcc, s_xccs;
    const int xcc = (int)(__builtin_amdgcn_s_getreg(kHwRegXccId) & (kMaxXcc - 1));
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(&counters[xcc * kLine], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&counters[kRegTotal * kLine], 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      (void)wait_counter<true>(counters, kRegTotal * kLine, (int)gridDim.x, ctl, limit);
      int xccs = 0;
      for (int x = 0; x < kMaxXcc; ++x) xccs += ld_relaxed(&counters[x * kLine]) > 0;
      s_on_xcc = ld_relaxed(&counters[xcc * kLine]);
      s_xccs = xccs;
    }
    __syncthreads();
    const int on_xcc = s_on_xcc, xccs = s_xccs;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    for (int L = 0; L < nlev; ++L) {
      if (threadIdx.x == 0) s_go = ld_relaxed(&ctl->abort) == 0;
      __syncthreads();
      const int lgo = __builtin_amdgcn_readfirstlane(s_go);
      __syncthreads();
      if (lgo && levels[L].parts) {
        // one (slot, panel, part) per workgroup, its entries split over
        // the four waves, whose minima meet in LDS; the workgroup takes the
        // next item of its XCD's range (longest first) whenever it is free
        const Level &lv = levels[L];
        const int k = __builtin_amdgcn_readfirstlane(lv.k);
        const int32_t nx = __builtin_amdgcn_readfirstlane(lv.nx);
        const int32_t x = (int32_t)blockIdx.x % nx;
        const int32_t x0 = __builtin_amdgcn_readfirstlane(lv.xr[x]);
        const int32_t count = __builtin_amdgcn_readfirstlane(lv.xr[x + 1]) - x0;
        const int32_t xbase = __builtin_amdgcn_readfirstlane(lv.xbase[x]);
        const kconst_u32 list = (kconst_u32)wave_uniform(items + lv.off + x0);
        while (true) {
          if (threadIdx.x == 0)
            s_task = __hip_atomic_fetch_add(&counters[(kTake + x) * kLine], 1, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT) - xbase;
          __syncthreads();
          const int32_t p = __builtin_amdgcn_readfirstlane(s_task);
          if (p >= count) break;
          // part_rows ends in a barrier: every wave has read s_task before
          // thread 0 writes the next
          part_item(slots, list[p], k, wv, lane, reinterpret_cast<uint32_t *>(lds));
        }
      } else if (lgo) {
        // A^1 (the only level of row items): row q, this lane's 8 columns,
        // from the masks; items dealt to the waves in turn
        const Level &lv = levels[L];
        const int64_t count = wave_uniform(lv.count);
        const kconst_u32 list = (kconst_u32)wave_uniform(items + lv.off);
        const int32_t W = (int32_t)gridDim.x * 4, w = (int32_t)blockIdx.x * 4 + wv;
        for (int64_t p = w; p < count; p += W) {
          const uint32_t code = list[p];
          const Slot &sl = slots[code >> 28];
          const int64_t N = wave_uniform((int64_t)sl.N), ld = wave_uniform(sl.ld);
          const uint32_t full = __builtin_amdgcn_readfirstlane(sl.full);
          const uint32_t *masks = wave_uniform(sl.masks);
          const int64_t panel = (code >> 20) & 0xFFu, q = code & 0xFFFFFu;
          const int64_t c0 = panel * kPanel + (int64_t)lane * 8;
          // lanes past the last column of the last panel store nothing
          if (c0 >= N) continue;
          const uint32_t mq = ((kconst_u32)masks)[q];
          uint32_t mp[8];
          if (c0 + 8 <= N) {
            const u32x4 lo = *(gconst<u32x4>)to_global(masks + c0);
            const u32x4 hi = *(gconst<u32x4>)to_global(masks + c0 + 4);
            mp[0] = lo.x; mp[1] = lo.y; mp[2] = lo.z; mp[3] = lo.w;
            mp[4] = hi.x; mp[5] = hi.y; mp[6] = hi.z; mp[7] = hi.w;
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) mp[j] = c0 + j < N ? masks[c0 + j] : 0u;
          }
          uint16_t e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            e[j] = (c0 + j < N && can_follow(mq, mp[j], full))
                       ? (uint16_t)__builtin_popcount(mp[j] & 0xFFFFu)
                       : kInf;
          uint16_t *row = wave_uniform(wave_uniform(sl.powers)[1]) + q * ld + c0;
          if (c0 + 8 <= N) {
            *(gmut<u32x4>)to_global_mut(row) = u32x4{
                (uint32_t)e[0] | ((uint32_t)e[1] << 16), (uint32_t)e[2] | ((uint32_t)e[3] << 16),
                (uint32_t)e[4] | ((uint32_t)e[5] << 16), (uint32_t)e[6] | ((uint32_t)e[7] << 16)};
          } else {
            for (int j = 0; j < 8 && c0 + j < N; ++j) row[j] = e[j];
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are in its L2
      __syncthreads();
      if (threadIdx.x == 0) {
        // a workgroup no longer on the XCC it registered on (moved by a wave
        // save and restore) writes its own L2 back: its XCC's leader cannot
        if ((int)(__builtin_amdgcn_s_getreg(kHwRegXccId) & (kMaxXcc - 1)) != xcc)
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int before = __hip_atomic_fetch_add(&counters[(kArrive + xcc) * kLine], 1,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1 == on_xcc * (L + 1)) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_fetch_add(&counters[kXccDone * kLine], 1, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          (void)wait_counter<true>(counters, kXccDone * kLine, xccs * (L + 1), ctl, limit);
          __hip_atomic_store(&counters[(kRelease + xcc) * kLine], L + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        } else {
          (void)wait_counter<true>(counters, (kRelease + xcc) * kLine, L + 1, ctl, limit);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
  }
  while (true) {
    if (threadIdx.x == 0) {
      int t = -1;
      for (int i = 0; i < kQueues && t < 0; ++i) {
        const int q = (home + i) % kQueues;
        const int cnt = ctl->qcnt[q];
        if (ld_relaxed(&ctl->head[q]) >= cnt) continue;
        const int k = atomicAdd(&ctl->head[q], 1);
        if (k < cnt) t = ctl->qbeg[q] + k;
      }
      int go = 0, fresh = 0;
      if (t >= 0) {
        go = ld_relaxed(&ctl->abort) == 0;
        const int d1 = tasks[t].dep, d2 = tasks[t].dep2;
        if (go) go = wait_counter(counters, d1, tasks[t].dep_target, ctl, limit);
        if (go) go = wait_counter(counters, d2, tasks[t].dep2_target, ctl, limit);
        fresh = (d1 != acq_dep || d2 != acq_dep2);
        acq_dep = d1;
        acq_dep2 = d2;
        // the powers this task reads are final once its counters are
        // complete; one acquire per new dependency makes them visible (it
        // invalidates the CU's L1, which the workgroup's waves share)
        if (go && fresh) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      s_task = t;
      s_go = go;
    }
    __syncthreads();
    // uniform across the workgroup: the task record is read with scalar loads
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    const int go = __builtin_amdgcn_readfirstlane(s_go);
    if (t < 0) break;
    const Task task = tasks[t];
    if (go) {
      const Slot sl = slots[task.slot];
      const int64_t N = sl.N, ld = sl.ld;
      if (task.type == kGemm && task.compact) {
        // (G_x + x) (G_y + y) = (G_x + l_x + G_y + l_y) + (x y - l_x - l_y),
        // l the factors' least residuals (final: a compact giant's tiles
        // wait for the whole of each factor): the residuals' product in 16
        // bits, lowered by l_x + l_y and stored as u8 (a clamped entry flags
        // the range); the tiles fold their least residual into the base's
        // second word.  Rebased so, a giant's residuals span what its own
        // entries span plus one product's gap, however deep its tree.
        const int64_t ld8 = sl.ld8;
        const int32_t *bx = sl.bases8[task.x], *by = sl.bases8[task.y];
        const int32_t lx = bx[1], ly = by[1];
        int32_t *bo = sl.bases8[task.out];
        gemm_tile<kGBM, kGBN, kGBK, 8, 8, uint8_t, true>(
            (int)N, (int)N, (int)N, sl.powers8[task.x], ld8, sl.powers8[task.y], ld8,
            sl.powers8[task.out], ld8, 0, task.row0, task.c0,
            reinterpret_cast<uint16_t(*)[kGBK][kGBM]>(lds),
            reinterpret_cast<uint16_t(*)[kGBK][kGBN]>(lds + 2 * kGBK * kGBM), ctl->status,
            (uint16_t)min(lx + ly, 0xFFFF), bo + 1);
        // every tile writes the same base word; readers see it through the
        // tile counters they wait for
        if (threadIdx.x == 0) bo[0] = bx[0] + lx + by[0] + ly;
      } else if (task.type == kGemm) {
        gemm_tile<kGBM, kGBN, kGBK, 8, 8, uint16_t, true>(
            (int)N, (int)N, (int)N, sl.powers[task.x], ld,
            sl.powers[task.y], ld, sl.powers[task.out], ld, 0, task.row0,
            task.c0,
            reinterpret_cast<uint16_t(*)[kGBK][kGBM]>(lds),
            reinterpret_cast<uint16_t(*)[kGBK][kGBN]>(lds + 2 * kGBK * kGBM));
      } else if (task.compact) {
        u16x2 acc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = splat(kInf);
        const int64_t ld8 = sl.ld8;
        for (int64_t k0 = 0; k0 < N; k0 += 64)
          trace_tile<uint8_t, true>(sl.powers8[task.x], ld8, sl.powers8[task.y], ld8, N,
                                    task.row0, k0, lds, acc);
        const int32_t best = block_min(acc, part);
        if (threadIdx.x == 0 && best < (int32_t)kInf)
          atomicMin(&results[task.inst], best + sl.bases8[task.x][0] + sl.bases8[task.y][0]);
      } else {
        u16x2 acc[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = splat(kInf);
        for (int64_t k0 = 0; k0 < N; k0 += 64)
          trace_tile<uint16_t, true>(sl.powers[task.x], ld,
                                     sl.powers[task.y], ld, N, task.row0,
                                     k0, lds, acc);
        const int32_t best = block_min(acc, part);
        if (threadIdx.x == 0 && best < (int32_t)kInf) atomicMin(&results[task.inst], best);
      }
      // a task others wait for: every wave's stores reach its L2 before the
      // workgroup's one release (an L2 write-back) and count
      if (task.done >= 0) __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();  // also keeps the LDS arena from being reused too early
    if (threadIdx.x == 0 && task.done >= 0) {
      __hip_atomic_fetch_add(&counters[task.done], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (task.done2 >= 0)
        __hip_atomic_fetch_add(&counters[task.done2], 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      if (task.done3 >= 0)
        __hip_atomic_fetch_add(&counters[task.done3], 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void fill_kernel(int32_t *p, int64_t count, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

// A buffer that has to grow is replaced by one at least twice its size and
// the old one is kept until the context is destroyed: hipFree and
// hipHostFree wait for the whole device, so freeing here would make a batch
// on this context wait for the batches other contexts have in flight.
hipError_t grow(Buf &b, size_t bytes, std::vector<void *> &retired) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  const size_t want = std::max(bytes, 2 * b.bytes);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) return e;
  if (b.p) retired.push_back(b.p);
  b.p = p;
  b.bytes = want;
  return hipSuccess;
}

hipError_t grow_host(Buf &b, size_t bytes, std::vector<void *> &retired) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  const size_t want = std::max(bytes, 2 * b.bytes);
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  if (b.p) retired.push_back(b.p);
  b.p = p;
  b.bytes = want;
  return hipSuccess;
}

// Keys of a power set: the exponent e for a 16-bit power, e + kCompactKey
// for a shared-base compact one, kTempKey and kTempKey + 1 for the two
// buffers a chain of giants steps through (in the set's chain form).
constexpr int kCompactKey = 1 << 16;
constexpr int kTempKey = 1 << 20;

struct PowerSet {
  int64_t N = 0, ld = 0;
  int c = 0;                 // baby steps (fixed at first use)
  // compact (fixed at first use): A^1 .. A^3 in 16 bits, A^3 on as u8
  // residuals over one base per power, rows of ld8 bytes, the two base words
  // after the residuals
  bool compact = false;
  int64_t ld8 = 0;
  // giants by continuing the chain (sparse steps) instead of dense products
  // (fixed at first use)
  bool chain_giants = false;
  std::map<int, void *> pw;  // key -> device buffer (inside a slab)
  std::set<int> have;        // keys known complete on the device
  std::vector<void *> slabs;  // one allocation per batch that added powers
  size_t held = 0;            // bytes of the slabs
  size_t bytes16() const { return (size_t)N * (size_t)ld * sizeof(uint16_t); }
  size_t bytes8() const { return (size_t)N * (size_t)ld8 + 256; }
  bool narrow(int key) const { return key >= kTempKey ? compact : key >= kCompactKey; }
  size_t bytes_of(int key) const { return narrow(key) ? bytes8() : bytes16(); }
  int32_t *base_of(int key) const {
    return (int32_t *)((char *)pw.at(key) + (size_t)N * (size_t)ld8);
  }
};

}  // namespace

struct Ctx {
  int device = 0;
  size_t budget = 0, used = 0;
  std::map<int, PowerSet> sets;
  Buf d_tasks, d_slots, d_ptrs, d_counters, d_results, d_ctl, d_levels, d_items;
  Buf h_tasks, h_slots, h_ptrs, h_ctl, h_levels, h_items;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  void *g_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t g_counter_cap = 0, g_result_cap = 0;
  int g_grid = 0;
  hipEvent_t staged = nullptr;
  // chain levels run on one stream per slot, between two events on the caller's stream
  hipStream_t chain_stream[kMaxSlots] = {nullptr};
  hipEvent_t chain_start = nullptr, chain_done[kMaxSlots] = {nullptr};
  int64_t wait_limit = 2000000000;  // 20 s at 100 MHz
  int baby[16] = {0};               // baby steps by n; 0 = automatic
  int compact_from = 10;            // path orders kept compact from A^3 on (0: none)
  int chain_giants_from = 10;       // path orders whose giants continue the chain (0: none)
  Buf d_status;                     // compact range flags since the last check
  int fused = 0;                    // chain levels inside the persistent launch
  int grid_override = 0;
  bool pending = false;                      // a batch was queued and not yet checked
  std::map<int, std::set<int>> pending_new;  // exponents that batch computes, by n
  // algorithmic work of the last batch queued: (min,+) operations of its
  // chain levels, dense products and traces, and their bytes (16-bit entries)
  double work_ops[3] = {0, 0, 0}, work_bytes = 0;
  // buffers and graphs replaced while the context lives, freed with it
  std::vector<void *> retired_dev, retired_host;
  std::vector<hipGraphExec_t> retired_exec;
  std::mutex mu;
};

namespace {

// Library-wide baby steps by n from the autotuner (0: none); a context's
// own parameter takes precedence.
std::mutex g_tune_mu;
int g_tuned_baby[2][16] = {{0}};  // [fused mode][n]

// Launches with level barriers need their whole grid resident at once; two of
// them running together on one device (batches of two contexts on two
// streams) could each hold part of the chip and wait for the rest until the
// wait limit.  Such launches are ordered one after another through one event
// per device (the end of the last one).
std::mutex g_barrier_mu;
std::map<int, hipEvent_t> g_barrier_done;

int auto_baby(int n) { return n >= 8 ? 16 : 32; }

// largest power of two <= j
int pow2_floor(int j) {
  int h = 1;
  while (h * 2 <= j) h *= 2;
  return h;
}

// the two giant indices whose product gives giant j (in units of c)
void giant_split(int j, int *l, int *r) {
  const int h = pow2_floor(j);
  if (h == j) {
    *l = j / 2;
    *r = j / 2;
  } else {
    *l = h;
    *r = j - h;
  }
}

// giant indices needed to build giant j (including j), into out
void giant_closure(int j, std::set<int> &out) {
  if (j <= 1 || out.count(j)) return;
  int l, r;
  giant_split(j, &l, &r);
  giant_closure(l, out);
  giant_closure(r, out);
  out.insert(j);
}

// The pair of exponents answering instance m with baby steps c: babies
// 1..c (1..c+2 for a compact set, whose pairs keep both exponents at 3 or
// above once one is: a compact power pairs only with a compact one).
void split_instance(int64_t m, int c, bool compact, int *a, int *b) {
  const int top = compact ? c + 2 : c;
  if (m <= 2 * (int64_t)top) {
    *a = (int)((m + 1) / 2);
    *b = (int)(m / 2);
  } else {
    const int lo = compact ? 3 : 1;  // the baby of the pair: lo .. top
    const int j = (int)((m - lo) / c);
    *a = j * c;
    *b = (int)(m - (int64_t)j * c);
  }
}

// whether the trace of the pair (a, b) reads compact powers
bool compact_pair(bool compact, int a, int b) { return compact && (a > 3 || b > 3); }

// Exponents a batch needs for one path order with baby steps c: the chain
// top and the giant indices (in units of c).
void batch_needs(const std::vector<int64_t> &ms, int c, bool compact, bool chain_giants,
                 int *chain_top, std::set<int> *giants) {
  const int top = compact ? c + 2 : c;
  *chain_top = 1;
  for (int64_t m : ms) {
    int a, b;
    split_instance(m, c, compact, &a, &b);
    if (m <= 2 * (int64_t)top) {
      *chain_top = std::max(*chain_top, a);
    } else {
      *chain_top = std::max(*chain_top, top);
      // a chained giant needs no smaller giants; a product giant its closure
      if (chain_giants)
        giants->insert(a / c);
      else
        giant_closure(a / c, *giants);
    }
  }
}

int capture_graph(Ctx *c, int grid) {
  if (c->exec) {
    // a batch queued earlier may still run it; destroyed with the context
    c->retired_exec.push_back(c->exec);
    c->exec = nullptr;
  }
  if (!c->cap_stream) TP_HIP_CHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  TP_HIP_CHECK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  const int64_t nc = (int64_t)(c->d_counters.bytes / sizeof(int32_t));
  const int64_t nr = (int64_t)(c->d_results.bytes / sizeof(int32_t));
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, c->cap_stream,
                     (int32_t *)c->d_counters.p, nc, 0);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, c->cap_stream,
                     (int32_t *)c->d_results.p, nr, (int32_t)kInf);
  hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(256), 0, c->cap_stream, (Control *)c->d_ctl.p,
                     (const Task *)c->d_tasks.p, (const Slot *)c->d_slots.p,
                     (const Level *)c->d_levels.p, (const uint32_t *)c->d_items.p,
                     (int32_t *)c->d_counters.p,
                     (int32_t *)c->d_results.p);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  c->g_key[0] = c->d_tasks.p;
  c->g_key[1] = c->d_counters.p;
  c->g_key[2] = c->d_results.p;
  c->g_key[3] = c->d_levels.p;
  c->g_key[4] = c->d_items.p;
  c->g_counter_cap = c->d_counters.bytes;
  c->g_result_cap = c->d_results.bytes;
  c->g_grid = grid;
  return TP_OK;
}

int default_grid() {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, 256, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 4;
  return cus * per_cu;
}

struct Plan {
  int n = 0, chain_top = 0;
  std::set<int> giants;   // giant indices (units of c)
  std::vector<int> exps;  // every exponent of the batch, increasing
  StateView view{};
  FineView fine{};        // fused mode: the row-block parts of the chain levels
};

int baby_of(Ctx *c, int n) {
  auto it = c->sets.find(n);
  if (it != c->sets.end() && it->second.c > 0) return it->second.c;
  if (c->baby[n] > 0) return c->baby[n];
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int t = g_tuned_baby[c->fused ? 1 : 0][n];
  return t > 0 ? t : auto_baby(n);
}

// Keys of the powers a batch needs for one path order (increasing): 16-bit
// A^1 .. A^top and the giants; for a compact set 16-bit A^1 .. A^3 and
// compact A^3 .. A^top and giants (when any pair or giant reads one).
std::vector<int> keys_of(int chain_top, const std::set<int> &giants, int c, bool compact,
                         bool chain_giants) {
  std::set<int> e;
  if (chain_giants && !giants.empty()) {
    e.insert(kTempKey);
    e.insert(kTempKey + 1);
  }
  if (!compact) {
    for (int k = 1; k <= chain_top; ++k) e.insert(k);
    for (int j : giants) e.insert(j * c);
  } else {
    for (int k = 1; k <= std::min(chain_top, 3); ++k) e.insert(k);
    if (chain_top >= 4 || !giants.empty())
      for (int k = 3; k <= chain_top; ++k) e.insert(k + kCompactKey);
    for (int j : giants) e.insert(j * c + kCompactKey);
  }
  return std::vector<int>(e.begin(), e.end());
}

// compact sets: at least 4 baby steps, so every giant factor is compact
int compact_baby(int c) { return std::max(c, 4); }

// Baby steps of a new set of path order n for the cycle orders ms of the
// batch that creates it: the tuned (or built-in) c0, or c1 = ceil(m_max / 2)
// when some cycle order needs giants at c0, c1 <= 2 c0 and the planner's
// rates put the extra c1 - c0 chain levels below the giants' products (c1
// answers every instance from two babies).  Baby steps set on the context,
// compact sets and chained giants keep c0.  `view` supplies the state's N
// and nnz when the choice needs them (it may build the state); a negative
// status from it is returned as is.
template <typename ViewFn>
int fresh_baby(Ctx *c, int n, const std::vector<int64_t> &ms, bool compact, bool chain_giants,
               ViewFn view) {
  const int c0 = compact ? compact_baby(baby_of(c, n)) : baby_of(c, n);
  if (compact || chain_giants || c->baby[n] > 0 || ms.empty()) return c0;
  const int64_t mmax = *std::max_element(ms.begin(), ms.end());
  if ((mmax + 1) / 2 > 2 * (int64_t)c0) return c0;
  const int c1 = (int)((mmax + 1) / 2);
  if (c1 <= c0) return c0;
  int top0 = 0;
  std::set<int> g0;
  batch_needs(ms, c0, false, false, &top0, &g0);
  if (g0.empty()) return c0;
  StateView v{};
  const int rc = view(&v);
  if (rc != TP_OK) return rc;
  double step = 0, product = 0;
  step_and_product_seconds(n, (double)v.N, (double)v.nnz, &step, &product);
  return (double)(c1 - top0) * step < (double)g0.size() * product ? c1 : c0;
}

// Baby steps of every path order of a batch (into *out): a resident set
// keeps its own; a new one takes fresh_baby's choice.  In fused mode, where
// the levels of every path order run together, a new 16-bit set that would
// still make giants chains to c1 = ceil(m_max / 2) instead when c1 is within
// the batch's deepest in-kernel chain (its levels run anyway).  view(n, v)
// supplies a state when a choice needs its cost.
template <typename ViewFn>
int plan_babies(Ctx *c, const std::map<int, std::vector<int64_t>> &by_n, ViewFn view,
                std::map<int, int> *out) {
  struct Form {
    bool fresh, compact, chain;
  };
  auto form_of = [&](int n) {
    auto it = c->sets.find(n);
    Form f{};
    f.fresh = it == c->sets.end() || it->second.c == 0;
    f.compact = f.fresh ? (c->compact_from > 0 && n >= c->compact_from && n >= 2)
                        : it->second.compact;
    f.chain = f.fresh ? (c->chain_giants_from > 0 && n >= c->chain_giants_from)
                      : it->second.chain_giants;
    return f;
  };
  int depth = 0;
  for (const auto &kv : by_n) {
    const int n = kv.first;
    const Form f = form_of(n);
    int cb = f.fresh ? fresh_baby(c, n, kv.second, f.compact, f.chain,
                                  [&](StateView *v) { return view(n, v); })
                     : c->sets[n].c;
    if (cb < 0) return cb;
    (*out)[n] = cb;
    if (c->fused && !f.compact && !f.chain) {
      int top = 0;
      std::set<int> g;
      batch_needs(kv.second, cb, false, false, &top, &g);
      depth = std::max(depth, top);
    }
  }
  if (!c->fused) return TP_OK;
  for (const auto &kv : by_n) {
    const int n = kv.first;
    const Form f = form_of(n);
    if (!f.fresh || f.compact || f.chain || c->baby[n] > 0) continue;
    const int64_t c1 = (*std::max_element(kv.second.begin(), kv.second.end()) + 1) / 2;
    if (c1 <= (*out)[n] || c1 > depth) continue;
    int top = 0;
    std::set<int> g;
    batch_needs(kv.second, (*out)[n], false, false, &top, &g);
    if (!g.empty()) (*out)[n] = (int)c1;
  }
  return TP_OK;
}

}  // namespace

namespace {

// Fused mode's level item lists.  A level k >= 2: (slot, panel, part)
// items in column order, cut into nx ranges of about equal work (a part's
// entry count plus the item's fixed cost, its start and its minima meeting
// in LDS, about 140 entries' worth at n = 9), each range longest first.
// Level 1: (slot, panel, row) items by decreasing length of the row's
// successor list (a bucket per out-degree), a row's panels together.  A list
// depends only on its slots' path orders and nx, so the process keeps those
// it built (g_lists).
struct LevelList {
  std::vector<uint32_t> items;
  Level cut{};
};
std::mutex g_list_mu;
std::map<std::vector<int>, LevelList> g_lists;  // (kind, nx, slot, n, slot, n, ...)

LevelList part_list(const std::vector<Plan> &plans, const std::vector<int> &set, int nx) {
  constexpr int64_t kItemCost = 140;
  std::vector<std::pair<int64_t, uint32_t>> its;
  for (int s : set) {
    const Plan &p = plans[s];
    const int64_t panels = (p.view.N + kPanel - 1) / kPanel;
    for (int64_t P = 0; P < panels; ++P)
      for (int64_t f = 0; f < p.fine.nf; ++f)
        its.push_back({p.fine.fptrh[f + 1] - p.fine.fptrh[f] + kItemCost, item_code(s, P, f)});
  }
  LevelList out;
  Level &cut = out.cut;
  cut.nx = nx;
  int64_t total = 0, acc = 0;
  for (const auto &x : its) total += x.first;
  int x = 1;
  for (size_t i = 0; i < its.size() && x < cut.nx; ++i) {
    acc += its[i].first;
    while (x < cut.nx && acc * cut.nx >= total * x) cut.xr[x++] = (int32_t)(i + 1);
  }
  for (; x <= cut.nx; ++x) cut.xr[x] = (int32_t)its.size();
  for (int r = 0; r < cut.nx; ++r)
    std::stable_sort(its.begin() + cut.xr[r], its.begin() + cut.xr[r + 1],
                     [](const std::pair<int64_t, uint32_t> &a,
                        const std::pair<int64_t, uint32_t> &b) { return a.first > b.first; });
  out.items.reserve(its.size());
  for (const auto &it : its) out.items.push_back(it.second);
  return out;
}

LevelList row_list(const std::vector<Plan> &plans, const std::vector<int> &set) {
  int maxdeg = 0;
  for (int s : set) {
    const Plan &p = plans[s];
    for (int64_t q = 0; q < p.view.N; ++q) maxdeg = std::max(maxdeg, (int)p.view.degh[q]);
  }
  std::vector<int64_t> pos((size_t)maxdeg + 1, 0);
  for (int s : set) {
    const Plan &p = plans[s];
    const int64_t panels = (p.view.N + kPanel - 1) / kPanel;
    for (int64_t q = 0; q < p.view.N; ++q) pos[p.view.degh[q]] += panels;
  }
  int64_t at = 0;
  for (int d = maxdeg; d >= 0; --d) {
    const int64_t n_d = pos[d];
    pos[d] = at;
    at += n_d;
  }
  LevelList out;
  out.items.resize((size_t)at);
  for (int s : set) {
    const Plan &p = plans[s];
    const int64_t panels = (p.view.N + kPanel - 1) / kPanel;
    for (int64_t q = 0; q < p.view.N; ++q)
      for (int64_t P = 0; P < panels; ++P)
        out.items[(size_t)pos[p.view.degh[q]]++] = item_code(s, P, q);
  }
  return out;
}

}  // namespace

int batch_run(Ctx *c, int count, const int32_t *ns, const int64_t *ms, int32_t *gamma2_dev,
              hipStream_t stream) {
  // wait until the previous batch's staging buffers have been consumed
  if (c->staged) TP_HIP_CHECK(hipEventSynchronize(c->staged));
  std::map<int, std::vector<int64_t>> by_n;
  for (int j = 0; j < count; ++j) by_n[ns[j]].push_back(ms[j]);
  TP_REQUIRE((int)by_n.size() <= kMaxSlots, "more than %d distinct n in one batch", kMaxSlots);

  std::map<int, int> babies;
  {
    const int rc = plan_babies(c, by_n,
                               [&](int n, StateView *v) { return state_view(n, stream, v); },
                               &babies);
    if (rc != TP_OK) return rc;
  }
  std::vector<Plan> plans;
  std::map<int, int> slot_of;
  int maxexp = 1;
  for (auto &kv : by_n) {
    Plan p;
    p.n = kv.first;
    const int rc = state_view(p.n, stream, &p.view);
    if (rc != TP_OK) return rc;
    PowerSet &ps = c->sets[p.n];
    ps.N = p.view.N;
    ps.ld = (p.view.N + 63) / 64 * 64;
    if (ps.c == 0) {
      // a new set: its form and baby steps are fixed now
      ps.compact = c->compact_from > 0 && p.n >= c->compact_from && p.n >= 2;
      ps.chain_giants = c->chain_giants_from > 0 && p.n >= c->chain_giants_from;
      ps.ld8 = (p.view.N + 63) / 64 * 64;
      ps.c = babies[p.n];
    }
    batch_needs(kv.second, ps.c, ps.compact, ps.chain_giants, &p.chain_top, &p.giants);
    p.exps = keys_of(p.chain_top, p.giants, ps.c, ps.compact, ps.chain_giants);
    for (int key : p.exps) maxexp = std::max(maxexp, key % kCompactKey);
    slot_of[p.n] = (int)plans.size();
    plans.push_back(p);
  }
  // memory: allocate every missing power, all or nothing
  {
    size_t extra = 0;
    for (const Plan &p : plans) {
      const PowerSet &ps = c->sets[p.n];
      for (int e : p.exps)
        if (!ps.pw.count(e)) extra += ps.bytes_of(e);
    }
    if (c->used + extra > c->budget) {
      set_error("batch needs %zu more bytes of resident powers; %zu of %zu bytes in use", extra,
                c->used, c->budget);
      return TP_ENOMEM;
    }
    // the new powers of one n in one allocation (a slab), cut in order
    for (const Plan &p : plans) {
      PowerSet &ps = c->sets[p.n];
      std::vector<int> missing;
      size_t total = 0;
      for (int e : p.exps)
        if (!ps.pw.count(e)) {
          missing.push_back(e);
          total += ps.bytes_of(e);  // multiples of 64 bytes
        }
      if (missing.empty()) continue;
      void *slab = nullptr;
      hipError_t err = hipMalloc(&slab, total);
      if (err != hipSuccess) return hip_fail(err, "hipMalloc (resident powers)");
      ps.slabs.push_back(slab);
      ps.held += total;
      c->used += total;
      size_t at = 0;
      for (int e : missing) {
        ps.pw[e] = (char *)slab + at;
        at += ps.bytes_of(e);
      }
    }
  }
  const int nslots = (int)plans.size();
  const bool fused = c->fused != 0;
  // missing chain levels of each slot: 16-bit k0[s] .. top16[s] (none if
  // beyond), and for a compact set compact k8[s] .. chain_top
  std::vector<int> k0(nslots), top16(nslots), k8(nslots);
  for (int s = 0; s < nslots; ++s) {
    const PowerSet &ps = c->sets[plans[s].n];
    top16[s] = ps.compact ? std::min(plans[s].chain_top, 3) : plans[s].chain_top;
    k0[s] = 1;
    while (k0[s] <= top16[s] && ps.have.count(k0[s])) ++k0[s];
    k8[s] = plans[s].chain_top + 1;
    if (ps.compact && ps.pw.count(3 + kCompactKey)) {
      k8[s] = 3;
      while (k8[s] <= plans[s].chain_top && ps.have.count(k8[s] + kCompactKey)) ++k8[s];
    }
  }
  // compact range flags (cleared by tp_ctx_check)
  if (!c->d_status.p) {
    TP_HIP_CHECK(grow(c->d_status, 256, c->retired_dev));
    TP_HIP_CHECK(launch_fill_i32((int32_t *)c->d_status.p, 1, 0, stream));
  }
  int32_t *status = (int32_t *)c->d_status.p;

  // the chain levels as plain launches (split mode, and the compact sets in
  // either mode), from the lowest missing level of each n up to its top, on
  // the slot's own stream after what the caller's stream has queued so far;
  // the caller's stream waits for them
  auto launched = [&](int s) {
    const PowerSet &ps = c->sets[plans[s].n];
    return !fused || ps.compact || ps.chain_giants;
  };
  // giants a chain makes: the missing ones of the sets that chain them
  std::vector<std::vector<int>> gchain(nslots);
  std::vector<int64_t> gsteps(nslots, 0);  // steps those chains take
  for (int s = 0; s < nslots; ++s) {
    const PowerSet &ps = c->sets[plans[s].n];
    if (!ps.chain_giants) continue;
    for (int j : plans[s].giants) {
      const int e = j * ps.c;
      if (!ps.have.count(ps.compact ? e + kCompactKey : e)) gchain[s].push_back(e);
    }
  }
  {
    bool any = false;
    for (int s = 0; s < nslots; ++s)
      any = any || (launched(s) && (k0[s] <= top16[s] || k8[s] <= plans[s].chain_top ||
                                    !gchain[s].empty()));
    if (any) {
      if (!c->chain_start)
        TP_HIP_CHECK(hipEventCreateWithFlags(&c->chain_start, hipEventDisableTiming));
      TP_HIP_CHECK(hipEventRecord(c->chain_start, stream));
    }
    // the chains in order of decreasing work, so the longest (the batch's
    // critical path) starts first and the host queues the others while it
    // runs; queued in slot order, the n = 9 chain of a mixed batch started
    // only after the smaller ones had been queued (about 1 ms later)
    std::vector<int> order(nslots);
    std::vector<double> work(nslots, 0.0);
    for (int s = 0; s < nslots; ++s) {
      order[s] = s;
      const int levels = std::max(0, top16[s] - k0[s] + 1) +
                         std::max(0, plans[s].chain_top - k8[s] + 1) +
                         (int)gchain[s].size() * c->sets[plans[s].n].c;
      work[s] = (double)levels * (double)plans[s].view.nnz * (double)plans[s].view.N;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    for (int s : order) {
      const Plan &p = plans[s];
      PowerSet &ps = c->sets[p.n];
      if (!launched(s) || (k0[s] > top16[s] && k8[s] > p.chain_top && gchain[s].empty()))
        continue;
      if (!c->chain_stream[s]) {
        TP_HIP_CHECK(hipStreamCreateWithFlags(&c->chain_stream[s], hipStreamNonBlocking));
        TP_HIP_CHECK(hipEventCreateWithFlags(&c->chain_done[s], hipEventDisableTiming));
      }
      hipStream_t cs = c->chain_stream[s];
      TP_HIP_CHECK(hipStreamWaitEvent(cs, c->chain_start, 0));
      for (int k = k0[s]; k <= top16[s]; ++k) {
        uint16_t *Y = (uint16_t *)ps.pw.at(k);
        if (k == 1)
          TP_HIP_CHECK(launch_dense_state(p.n, ps.N, p.view.masks, TP_U16, Y, ps.ld, cs));
        else
          TP_HIP_CHECK(state_step_view(p.view, (const uint16_t *)ps.pw.at(k - 1), ps.ld, Y,
                                       ps.ld, ps.N, cs));
      }
      for (int k = k8[s]; k <= p.chain_top; ++k) {
        uint8_t *Y = (uint8_t *)ps.pw.at(k + kCompactKey);
        int32_t *by = ps.base_of(k + kCompactKey);
        if (k == 3)
          TP_HIP_CHECK(launch_shared_from_u16(ps.N, ps.N, (const uint16_t *)ps.pw.at(3), ps.ld, Y,
                                              ps.ld8, by, status, cs));
        else
          TP_HIP_CHECK(launch_shared_step(p.view, (const uint8_t *)ps.pw.at(k - 1 + kCompactKey),
                                          ps.ld8, ps.base_of(k - 1 + kCompactKey), Y, ps.ld8, by,
                                          ps.N, status, cs));
      }
      // giants by continuing the chain: from the highest power below each
      // missing giant (the babies' top, a resident giant or the last one
      // made), through the two step buffers, into the giant
      if (!gchain[s].empty()) {
        const int top = p.chain_top;
        auto form_key = [&](int e) { return ps.compact ? e + kCompactKey : e; };
        int from = top;  // the babies' top is complete on this stream
        for (int e : gchain[s]) {
          for (const auto &kv : ps.pw) {
            const int k = kv.first;
            if (k >= kTempKey || (ps.compact != (k >= kCompactKey))) continue;
            const int ek = k % kCompactKey;
            if (ek < e && ek > from && ps.have.count(k)) from = ek;
          }
          gsteps[s] += e - from;
          for (int k = from + 1; k <= e; ++k) {
            const int xk = k - 1 == from ? form_key(from) : kTempKey + ((k - 1) & 1);
            const int yk = k == e ? form_key(e) : kTempKey + (k & 1);
            if (ps.compact)
              TP_HIP_CHECK(launch_shared_step(p.view, (const uint8_t *)ps.pw.at(xk), ps.ld8,
                                              ps.base_of(xk), (uint8_t *)ps.pw.at(yk), ps.ld8,
                                              ps.base_of(yk), ps.N, status, cs));
            else
              TP_HIP_CHECK(state_step_view(p.view, (const uint16_t *)ps.pw.at(xk), ps.ld,
                                           (uint16_t *)ps.pw.at(yk), ps.ld, ps.N, cs));
          }
          from = e;
        }
      }
      TP_HIP_CHECK(hipEventRecord(c->chain_done[s], cs));
      TP_HIP_CHECK(hipStreamWaitEvent(stream, c->chain_done[s], 0));
    }
  }

  // fused mode: the missing chain levels as a level table the persistent
  // kernel runs first, level k over every slot that lacks A^k; each level
  // ends in a barrier over the grid, so the tasks below see complete powers
  // in both modes
  std::vector<Level> levels;
  std::vector<uint32_t> items;
  // one level item list (its items appended to `items`, at *off, *cnt),
  // from the process's cache when these slots held these path orders before
  auto add_list = [&](int kind, const std::vector<int> &set, int nx, Level *cut, int64_t *off,
                      int64_t *cnt) {
    std::vector<int> key{kind, nx};
    for (int s : set) {
      key.push_back(s);
      key.push_back(plans[s].n);
    }
    std::lock_guard<std::mutex> lk(g_list_mu);
    auto it = g_lists.find(key);
    if (it == g_lists.end()) {
      if (g_lists.size() >= 256) g_lists.clear();
      it = g_lists.emplace(key, kind == 1 ? row_list(plans, set) : part_list(plans, set, nx)).first;
    }
    *off = (int64_t)items.size();
    *cnt = (int64_t)it->second.items.size();
    items.insert(items.end(), it->second.items.begin(), it->second.items.end());
    *cut = it->second.cut;
  };
  // the grid of a launch with levels (every workgroup resident)
  const int resident = default_grid();
  const int grid_levels =
      c->grid_override > 0 ? std::min(c->grid_override, resident) : resident;
  if (fused) {
    int max_top = 0;
    for (const Plan &p : plans) max_top = std::max(max_top, p.chain_top);
    for (int s = 0; s < nslots; ++s) {
      if (launched(s) || plans[s].chain_top < std::max(k0[s], 2)) continue;
      const int rc = state_fine_view(plans[s].n, stream, &plans[s].fine);
      if (rc != TP_OK) return rc;
    }
    int32_t xbase[kXcds] = {0};
    std::vector<int> prev_set, prev_part_set;
    int64_t off = 0, cnt = 0, part_off = 0, part_cnt = 0;
    Level part_cut{};
    for (int k = 1; k <= max_top; ++k) {
      std::vector<int> set;
      for (int s = 0; s < nslots; ++s)
        if (!launched(s) && k >= k0[s] && k <= plans[s].chain_top) set.push_back(s);
      if (set.empty()) continue;
      if (k >= 2) {
        if (set != prev_part_set) {
          add_list(2, set, std::max(1, std::min(kXcds, grid_levels)), &part_cut, &part_off,
                   &part_cnt);
          prev_part_set = set;
        }
        Level lv = part_cut;
        lv.k = k;
        lv.parts = 1;
        lv.off = part_off;
        lv.count = part_cnt;
        for (int x = 0; x < lv.nx; ++x) {
          lv.xbase[x] = xbase[x];
          xbase[x] += lv.xr[x + 1] - lv.xr[x] + (grid_levels - 1 - x) / lv.nx + 1;
        }
        levels.push_back(lv);
        continue;
      }
      if (set != prev_set) {
        Level unused{};
        add_list(1, set, 0, &unused, &off, &cnt);
        prev_set = set;
      }
      Level lv{};
      lv.k = k;
      lv.off = off;
      lv.count = cnt;
      levels.push_back(lv);
    }
  }
  // completion counters: the level barriers first, then the giants (one per
  // 128-row block and one per 128-column block)
  const int ncounters0 = levels.empty() ? 0 : kLevelCounters;
  int ncounters = 0;
  std::map<std::pair<int, int>, int> gbase;
  std::vector<int> nblk(nslots);
  for (int s = 0; s < nslots; ++s) {
    const PowerSet &ps = c->sets[plans[s].n];
    nblk[s] = (int)((ps.N + kGBM - 1) / kGBM);
    for (int j : plans[s].giants) {
      const int e = j * ps.c;
      if (ps.chain_giants) continue;  // made by the chain before the kernel
      if (ps.have.count(ps.compact ? e + kCompactKey : e)) continue;
      gbase[{s, e}] = ncounters;
      // a compact giant also counts its finished tiles in all: the tiles of
      // a giant made from it wait for the whole of it (its least residual)
      ncounters += 2 * nblk[s] + (ps.compact ? 1 : 0);
    }
  }
  // a new compact giant's least residual starts above any residual; its
  // tiles lower it
  for (const auto &kv : gbase) {
    const PowerSet &ps = c->sets[plans[kv.first.first].n];
    if (ps.compact)
      TP_HIP_CHECK(launch_fill_i32(ps.base_of(kv.first.second + kCompactKey) + 1, 1, 0x7FFFFFFF,
                                   stream));
  }
  auto is_new_giant = [&](int s, int e) { return gbase.count({s, e}) != 0; };
  auto pending = [&](int s, int e) { return is_new_giant(s, e); };

  // the batch's algorithmic work: a chain level nnz(A) * N operations over
  // 4 N^2 bytes (X read, Y written), a dense product N^3 over 6 N^2, a trace
  // N^2 over 4 N^2
  c->work_ops[0] = c->work_ops[1] = c->work_ops[2] = 0;
  c->work_bytes = 0;
  for (int s = 0; s < nslots; ++s) {
    const double N = (double)plans[s].view.N, nnz = (double)plans[s].view.nnz;
    for (int k = std::max(k0[s], 2); k <= top16[s]; ++k) {
      c->work_ops[0] += nnz * N;
      c->work_bytes += 4 * N * N;
    }
    for (int k = std::max(k8[s], 4); k <= plans[s].chain_top; ++k) {  // compact steps
      c->work_ops[0] += nnz * N;
      c->work_bytes += 4 * N * N;
    }
    c->work_ops[0] += (double)gsteps[s] * nnz * N;  // chained giants
    c->work_bytes += (double)gsteps[s] * 4 * N * N;
    if (k0[s] <= 1 && plans[s].chain_top >= 1) c->work_bytes += 2 * N * N;  // A^1 written
  }
  for (const auto &kv : gbase) {
    const double N = (double)plans[kv.first.first].view.N;
    c->work_ops[1] += N * N * N;
    c->work_bytes += 6 * N * N;
  }
  for (int j = 0; j < count; ++j) {
    const double N = (double)plans[slot_of[ns[j]]].view.N;
    c->work_ops[2] += N * N;
    c->work_bytes += 4 * N * N;
  }

  std::vector<Task> tasks;
  // dependency on rows [r0, r0 + 128) (all columns) of exponent e
  auto rows_dep = [&](int s, int e, int64_t r0, int32_t *dep, int32_t *target) {
    auto it = gbase.find({s, e});
    if (it != gbase.end()) {
      *dep = it->second + (int)(r0 / kGBM);
      *target = nblk[s];
    } else {
      *dep = -1;
      *target = 0;
    }
  };
  // dependency on columns [c0, c0 + 128) (all rows) of exponent e
  auto cols_dep = [&](int s, int e, int64_t c0, int32_t *dep, int32_t *target) {
    auto it = gbase.find({s, e});
    if (it != gbase.end()) {
      *dep = it->second + nblk[s] + (int)(c0 / kGBN);
      *target = nblk[s];
    } else {
      rows_dep(s, e, 0, dep, target);
    }
  };

  // a group of tasks (one giant product or one instance's traces) is dealt to
  // the queues in contiguous chunks, so that the tasks an XCD runs together
  // share their inputs in its L2
  auto deal = [&](size_t first) {
    const size_t cnt = tasks.size() - first;
    for (size_t i = 0; i < cnt; ++i) tasks[first + i].queue = (int32_t)(i * kQueues / cnt);
  };

  // every instance's pair of exponents; traces are queued right after the
  // last power they read
  std::vector<int> ta(count), tb(count);
  std::vector<std::vector<int>> waiting(nslots);
  for (int j = 0; j < count; ++j) {
    const int s = slot_of[ns[j]];
    split_instance(ms[j], c->sets[ns[j]].c, c->sets[ns[j]].compact, &ta[j], &tb[j]);
    waiting[s].push_back(j);
  }
  auto push_ready_traces = [&](int s, int upto) {
    std::vector<int> rest;
    for (int j : waiting[s]) {
      const int a = ta[j], b = tb[j];
      const bool ready = (!pending(s, a) || a <= upto) && (!pending(s, b) || b <= upto);
      if (!ready) {
        rest.push_back(j);
        continue;
      }
      const int64_t N = c->sets[plans[s].n].N;
      const size_t first = tasks.size();
      for (int64_t i0 = 0; i0 < N; i0 += 64) {
        Task t{};
        t.type = kTrace;
        t.slot = s;
        t.x = a;
        t.y = b;
        t.row0 = (int32_t)i0;
        t.row1 = (int32_t)std::min<int64_t>(i0 + 64, N);
        rows_dep(s, a, i0, &t.dep, &t.dep_target);
        cols_dep(s, b, i0, &t.dep2, &t.dep2_target);
        t.done = t.done2 = t.done3 = -1;
        t.inst = j;
        t.compact = compact_pair(c->sets[plans[s].n].compact, a, b);
        tasks.push_back(t);
      }
      deal(first);
    }
    waiting[s].swap(rest);
  };

  // instances answered by powers complete before the launch first
  for (int s = 0; s < nslots; ++s) push_ready_traces(s, 0);

  // giants in increasing exponent, interleaved over n; a giant's two factors
  // have smaller exponents and are queued before it
  std::vector<std::vector<int>> gl(nslots);
  size_t rounds = 0;
  for (int s = 0; s < nslots; ++s) {
    gl[s].assign(plans[s].giants.begin(), plans[s].giants.end());
    rounds = std::max(rounds, gl[s].size());
  }
  for (size_t r = 0; r < rounds; ++r) {
    for (int s = 0; s < nslots; ++s) {
      if (r >= gl[s].size()) continue;
      const PowerSet &ps = c->sets[plans[s].n];
      const int j = gl[s][r], e = j * ps.c;
      if (is_new_giant(s, e)) {
        int l, rr;
        giant_split(j, &l, &rr);
        const int x = l * ps.c, y = rr * ps.c;
        const size_t first = tasks.size();
        for (int64_t m0 = 0; m0 < ps.N; m0 += kGBM) {
          for (int64_t n0 = 0; n0 < ps.N; n0 += kGBN) {
            Task t{};
            t.type = kGemm;
            t.slot = s;
            t.out = e;
            t.x = x;
            t.y = y;
            t.row0 = (int32_t)m0;
            t.c0 = (int32_t)n0;
            t.done = gbase.at({s, e}) + (int)(m0 / kGBM);
            t.done2 = gbase.at({s, e}) + nblk[s] + (int)(n0 / kGBN);
            t.done3 = -1;
            t.compact = ps.compact;
            if (ps.compact) {
              // the whole of each factor that is a new giant
              const int32_t all = nblk[s] * nblk[s];
              t.dep = is_new_giant(s, x) ? gbase.at({s, x}) + 2 * nblk[s] : -1;
              t.dep_target = t.dep >= 0 ? all : 0;
              t.dep2 = is_new_giant(s, y) ? gbase.at({s, y}) + 2 * nblk[s] : -1;
              t.dep2_target = t.dep2 >= 0 ? all : 0;
              t.done3 = gbase.at({s, e}) + 2 * nblk[s];
            } else {
              rows_dep(s, x, m0, &t.dep, &t.dep_target);
              cols_dep(s, y, n0, &t.dep2, &t.dep2_target);
            }
            tasks.push_back(t);
          }
        }
        deal(first);
      }
      push_ready_traces(s, e);
    }
  }
  for (int s = 0; s < nslots; ++s) push_ready_traces(s, maxexp);
  for (int s = 0; s < nslots; ++s)
    if (!waiting[s].empty()) {
      set_error("internal: an instance of n = %d has no plan", plans[s].n);
      return TP_EINVAL;
    }

  // counters in memory: the level barrier's first, then one 256-byte line
  // per task counter (atomics and polls on one line serialize)
  const int cfirst = ncounters0;
  auto phys = [&](int32_t ix) { return ix < 0 ? ix : (int32_t)(cfirst + ix * kLine); };
  for (Task &t : tasks) {
    t.dep = phys(t.dep);
    t.dep2 = phys(t.dep2);
    t.done = phys(t.done);
    t.done2 = phys(t.done2);
    t.done3 = phys(t.done3);
  }
  const int64_t counter_words = (int64_t)cfirst + (int64_t)ncounters * kLine;

  // queues: each keeps the dependency order of the whole list
  std::vector<Task> ordered;
  ordered.reserve(tasks.size());
  int32_t qbeg[kQueues], qcnt[kQueues];
  for (int q = 0; q < kQueues; ++q) {
    qbeg[q] = (int32_t)ordered.size();
    for (const Task &t : tasks)
      if (t.queue == q) ordered.push_back(t);
    qcnt[q] = (int32_t)ordered.size() - qbeg[q];
  }
  tasks.swap(ordered);

  // staging (pinned) and device buffers
  const size_t tbytes = tasks.size() * sizeof(Task);
  // per slot three tables by exponent: 16-bit powers, compact residuals,
  // compact base words
  const size_t ptr_stride = (size_t)maxexp + 1;
  const size_t nptr = 3 * ptr_stride * nslots;
  TP_HIP_CHECK(grow_host(c->h_tasks, std::max<size_t>(tbytes, sizeof(Task)), c->retired_host));
  TP_HIP_CHECK(grow_host(c->h_slots, kMaxSlots * sizeof(Slot), c->retired_host));
  TP_HIP_CHECK(grow_host(c->h_ptrs, nptr * sizeof(void *), c->retired_host));
  TP_HIP_CHECK(grow_host(c->h_ctl, sizeof(Control), c->retired_host));
  TP_HIP_CHECK(grow(c->d_tasks, std::max<size_t>(tbytes, sizeof(Task)), c->retired_dev));
  TP_HIP_CHECK(grow(c->d_slots, kMaxSlots * sizeof(Slot), c->retired_dev));
  TP_HIP_CHECK(grow(c->d_ptrs, nptr * sizeof(void *), c->retired_dev));
  TP_HIP_CHECK(grow(c->d_ctl, sizeof(Control), c->retired_dev));
  TP_HIP_CHECK(grow(c->d_counters, (size_t)std::max<int64_t>(counter_words, 1) * sizeof(int32_t),
                    c->retired_dev));
  TP_HIP_CHECK(grow(c->d_results, (size_t)std::max(count, 1) * sizeof(int32_t), c->retired_dev));
  const size_t lbytes = levels.size() * sizeof(Level);
  const size_t ibytes = items.size() * sizeof(uint32_t);
  if (lbytes) {
    TP_HIP_CHECK(grow_host(c->h_levels, lbytes, c->retired_host));
    TP_HIP_CHECK(grow(c->d_levels, lbytes, c->retired_dev));
    memcpy(c->h_levels.p, levels.data(), lbytes);
    TP_HIP_CHECK(grow_host(c->h_items, ibytes, c->retired_host));
    TP_HIP_CHECK(grow(c->d_items, ibytes, c->retired_dev));
    memcpy(c->h_items.p, items.data(), ibytes);
  }

  memcpy(c->h_tasks.p, tasks.data(), tbytes);
  Slot *hs = (Slot *)c->h_slots.p;
  void **hp = (void **)c->h_ptrs.p;
  for (int s = 0; s < nslots; ++s) {
    const Plan &p = plans[s];
    const PowerSet &ps = c->sets[p.n];
    Slot sl{};
    sl.n = p.n;
    sl.N = (int32_t)ps.N;
    sl.ld = ps.ld;
    sl.full = (1u << p.n) - 1u;
    sl.masks = p.view.masks;
    sl.rowptr = p.view.rowptr;
    sl.colz = p.view.colz;
    void **tab = (void **)c->d_ptrs.p + 3 * ptr_stride * s;
    sl.powers = (uint16_t *const *)tab;
    sl.ld8 = ps.ld8;
    sl.powers8 = (uint8_t *const *)(tab + ptr_stride);
    sl.bases8 = (int32_t *const *)(tab + 2 * ptr_stride);
    sl.fptr = p.fine.fptr;
    sl.fent = p.fine.fent;
    sl.finfo = p.fine.finfo;
    hs[s] = sl;
    void **htab = hp + 3 * ptr_stride * s;
    for (size_t e = 0; e < ptr_stride; ++e) {
      auto it = ps.pw.find((int)e);
      htab[e] = it == ps.pw.end() ? nullptr : it->second;
      auto it8 = ps.pw.find((int)e + kCompactKey);
      htab[ptr_stride + e] = it8 == ps.pw.end() ? nullptr : it8->second;
      htab[2 * ptr_stride + e] = it8 == ps.pw.end() ? nullptr : ps.base_of((int)e + kCompactKey);
    }
  }
  Control *hc = (Control *)c->h_ctl.p;
  for (int q = 0; q < kQueues; ++q) {
    hc->head[q] = 0;
    hc->qbeg[q] = qbeg[q];
    hc->qcnt[q] = qcnt[q];
  }
  hc->abort = 0;
  hc->nlevels = (int32_t)levels.size();
  hc->wait_limit = c->wait_limit;
  hc->status = status;

  // the level barriers need every workgroup resident at once: a fused batch
  // with chain levels never launches more than the chip holds
  int grid = c->grid_override > 0 ? c->grid_override : resident;
  if (!levels.empty()) grid = grid_levels;
  if (!c->exec || c->g_key[0] != c->d_tasks.p || c->g_key[1] != c->d_counters.p ||
      c->g_key[2] != c->d_results.p || c->g_key[3] != c->d_levels.p ||
      c->g_key[4] != c->d_items.p || c->g_grid != grid ||
      c->g_counter_cap != c->d_counters.bytes || c->g_result_cap != c->d_results.bytes) {
    const int rc = capture_graph(c, grid);
    if (rc != TP_OK) return rc;
  }
  TP_HIP_CHECK(hipMemcpyAsync(c->d_tasks.p, c->h_tasks.p, tbytes, hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_slots.p, c->h_slots.p, nslots * sizeof(Slot),
                              hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_ptrs.p, c->h_ptrs.p, nptr * sizeof(void *),
                              hipMemcpyHostToDevice, stream));
  TP_HIP_CHECK(hipMemcpyAsync(c->d_ctl.p, c->h_ctl.p, sizeof(Control), hipMemcpyHostToDevice,
                              stream));
  if (lbytes) {
    TP_HIP_CHECK(hipMemcpyAsync(c->d_levels.p, c->h_levels.p, lbytes, hipMemcpyHostToDevice,
                                stream));
    TP_HIP_CHECK(hipMemcpyAsync(c->d_items.p, c->h_items.p, ibytes, hipMemcpyHostToDevice,
                                stream));
  }
  if (!c->staged) TP_HIP_CHECK(hipEventCreateWithFlags(&c->staged, hipEventDisableTiming));
  TP_HIP_CHECK(hipEventRecord(c->staged, stream));
  if (levels.empty()) {
    TP_HIP_CHECK(hipGraphLaunch(c->exec, stream));
  } else {
    std::lock_guard<std::mutex> lk(g_barrier_mu);
    hipEvent_t &done = g_barrier_done[c->device];
    if (done)
      TP_HIP_CHECK(hipStreamWaitEvent(stream, done, 0));
    else
      TP_HIP_CHECK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    TP_HIP_CHECK(hipGraphLaunch(c->exec, stream));
    TP_HIP_CHECK(hipEventRecord(done, stream));
  }
  TP_HIP_CHECK(hipMemcpyAsync(gamma2_dev, c->d_results.p, (size_t)count * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, stream));
  // what this batch computes counts as resident for later batches on this
  // stream; tp_ctx_check drops it again if the batch aborted
  c->pending = true;
  for (const Plan &p : plans) {
    PowerSet &ps = c->sets[p.n];
    for (int e : p.exps)
      if (!ps.have.count(e)) {
        ps.have.insert(e);
        c->pending_new[p.n].insert(e);
      }
  }
  return TP_OK;
}

int ctx_check(Ctx *c, hipStream_t stream) {
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  if (!c->pending) return TP_OK;
  c->pending = false;
  int32_t abort = 0;
  if (c->d_ctl.p) {
    // on the batch's stream (a synchronous copy would also wait for other
    // contexts' batches)
    TP_HIP_CHECK(hipMemcpyAsync(&abort, (char *)c->d_ctl.p + offsetof(Control, abort),
                                sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    TP_HIP_CHECK(hipStreamSynchronize(stream));
  }
  int32_t range = 0;
  if (c->d_status.p) {
    TP_HIP_CHECK(hipMemcpyAsync(&range, c->d_status.p, sizeof(int32_t), hipMemcpyDeviceToHost,
                                stream));
    TP_HIP_CHECK(hipStreamSynchronize(stream));
    if (range) {
      TP_HIP_CHECK(launch_fill_i32((int32_t *)c->d_status.p, 1, 0, stream));
      TP_HIP_CHECK(hipStreamSynchronize(stream));
    }
  }
  if (abort || range) {
    // nothing the failed batches were to compute can be trusted
    for (auto &kv : c->pending_new)
      for (int e : kv.second) c->sets[kv.first].have.erase(e);
    c->pending_new.clear();
    if (abort) {
      set_error("batch aborted: a task waited longer than the limit for its inputs");
      return TP_ECANCELED;
    }
    set_error("a compact power left the range of its 8-bit residuals");
    return TP_EOVERFLOW;
  }
  c->pending_new.clear();
  return TP_OK;
}

void ctx_free(Ctx *c) {
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->staged) (void)hipEventDestroy(c->staged);
  if (c->chain_start) (void)hipEventDestroy(c->chain_start);
  for (int s = 0; s < kMaxSlots; ++s) {
    if (c->chain_done[s]) (void)hipEventDestroy(c->chain_done[s]);
    if (c->chain_stream[s]) (void)hipStreamDestroy(c->chain_stream[s]);
  }
  for (auto &kv : c->sets)
    for (void *slab : kv.second.slabs) (void)hipFree(slab);
  Buf *dev[] = {&c->d_tasks, &c->d_slots,  &c->d_ptrs,   &c->d_counters,
                &c->d_results, &c->d_ctl, &c->d_levels, &c->d_items};
  for (Buf *b : dev)
    if (b->p) (void)hipFree(b->p);
  Buf *host[] = {&c->h_tasks, &c->h_slots, &c->h_ptrs, &c->h_ctl, &c->h_levels, &c->h_items};
  for (Buf *b : host)
    if (b->p) (void)hipHostFree(b->p);
  for (hipGraphExec_t g : c->retired_exec) (void)hipGraphExecDestroy(g);
  for (void *p : c->retired_dev) (void)hipFree(p);
  for (void *p : c->retired_host) (void)hipHostFree(p);
}

}  // namespace tp

using namespace tp;

extern "C" {

int tp_ctx_create(size_t hbm_budget_bytes, void **ctx) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = new Ctx();
  (void)hipGetDevice(&c->device);
  c->budget = hbm_budget_bytes;
  *ctx = c;
  return TP_OK;
}

int tp_ctx_destroy(void *ctx) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    (void)hipDeviceSynchronize();
    ctx_free(c);
  }
  delete c;
  return TP_OK;
}

int tp_ctx_set_param(void *ctx, int param, int64_t value) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (param == TP_PARAM_WAIT_LIMIT_US) {
    TP_REQUIRE(value >= 0, "negative wait limit");
    c->wait_limit = value * 100;  // 100 MHz ticks
    return TP_OK;
  }
  if (param == TP_PARAM_GRID) {
    // every queue needs a home workgroup (see the kernel): at least 8
    TP_REQUIRE(value == 0 || (value >= kQueues && value <= (1 << 20)),
               "grid must be 0 (fill the chip) or in %d..%d", kQueues, 1 << 20);
    c->grid_override = (int)value;
    return TP_OK;
  }
  if (param == TP_PARAM_FUSED_CHAIN) {
    TP_REQUIRE(value == 0 || value == 1, "TP_PARAM_FUSED_CHAIN is 0 or 1");
    c->fused = (int)value;
    return TP_OK;
  }
  if (param == TP_PARAM_CHAIN_GIANTS_FROM) {
    TP_REQUIRE(value >= 0 && value <= 13,
               "TP_PARAM_CHAIN_GIANTS_FROM is 0 (never) or a path order");
    for (auto &kv : c->sets)
      TP_REQUIRE(kv.second.pw.empty() ||
                     kv.second.chain_giants == (value > 0 && kv.first >= value),
                 "how n = %d makes its giants is fixed once its powers are resident", kv.first);
    c->chain_giants_from = (int)value;
    return TP_OK;
  }
  if (param == TP_PARAM_COMPACT_FROM) {
    TP_REQUIRE(value >= 0 && value <= 13, "TP_PARAM_COMPACT_FROM is 0 (never) or a path order");
    for (auto &kv : c->sets)
      TP_REQUIRE(kv.second.pw.empty() || kv.second.compact == (value > 0 && kv.first >= value &&
                                                               kv.first >= 2),
                 "the form of n = %d is fixed once its powers are resident", kv.first);
    c->compact_from = (int)value;
    return TP_OK;
  }
  if (param >= TP_PARAM_BABY_STEPS && param < TP_PARAM_BABY_STEPS + 16) {
    const int n = param - TP_PARAM_BABY_STEPS;
    TP_REQUIRE(value >= 0 && value <= (1 << 16), "baby steps out of range");
    TP_REQUIRE(c->sets.count(n) == 0 || c->sets[n].pw.empty(),
               "baby steps of n = %d are fixed once powers are resident", n);
    c->baby[n] = (int)value;
    return TP_OK;
  }
  set_error("unknown parameter %d", param);
  return TP_EINVAL;
}

int64_t tp_ctx_resident_bytes(void *ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return TP_EINVAL;
  }
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  return (int64_t)c->used;
}

int tp_ctx_release(void *ctx, int n, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  TP_REQUIRE(n >= 0 && n <= 12, "n = %d outside 0..12", n);
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  // queued batches may still read the powers
  TP_HIP_CHECK(hipStreamSynchronize(stream));
  for (auto it = c->sets.begin(); it != c->sets.end();) {
    if (n != 0 && it->first != n) {
      ++it;
      continue;
    }
    for (void *slab : it->second.slabs) TP_HIP_CHECK(hipFree(slab));
    c->used -= it->second.held;
    c->pending_new.erase(it->first);
    it = c->sets.erase(it);
  }
  return TP_OK;
}

int tp_ctx_copy_power(void *ctx, int n, int e, void *d_out, int64_t ld, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  TP_REQUIRE(d_out != nullptr, "out is NULL");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->sets.find(n);
  TP_REQUIRE(e >= 1 && e < kCompactKey, "no power %d", e);
  const bool have16 = it != c->sets.end() && it->second.have.count(e) && it->second.pw.count(e);
  const int k8 = e + kCompactKey;
  const bool have8 = it != c->sets.end() && it->second.have.count(k8) && it->second.pw.count(k8);
  TP_REQUIRE(have16 || have8, "the context holds no power %d of A(D_%d)", e, n);
  const PowerSet &ps = it->second;
  TP_REQUIRE(ld >= ps.N, "ld = %lld < N = %lld", (long long)ld, (long long)ps.N);
  if (ps.N == 0) return TP_OK;
  if (!have16) {
    // a compact power: base + residual, expanded to 16 bits
    TP_HIP_CHECK(launch_shared_to_u16(ps.N, ps.N, (const uint8_t *)ps.pw.at(k8), ps.ld8,
                                      ps.base_of(k8), (uint16_t *)d_out, ld, stream));
    return TP_OK;
  }
  TP_HIP_CHECK(hipMemcpy2DAsync(d_out, (size_t)ld * sizeof(uint16_t), ps.pw.at(e),
                                (size_t)ps.ld * sizeof(uint16_t), (size_t)ps.N * sizeof(uint16_t),
                                (size_t)ps.N, hipMemcpyDeviceToDevice, stream));
  return TP_OK;
}

int64_t tp_ctx_need_bytes(void *ctx, int count, const int32_t *n, const int64_t *m) {
  if (!ctx || count < 0 || (count > 0 && (!n || !m))) {
    set_error("bad arguments");
    return TP_EINVAL;
  }
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  std::map<int, std::vector<int64_t>> by_n;
  for (int j = 0; j < count; ++j) {
    if (n[j] < 1 || n[j] > 12 || m[j] < 3) {
      set_error("instance %d out of range", j);
      return TP_EINVAL;
    }
    by_n[n[j]].push_back(m[j]);
  }
  // the states are built now if a choice of baby steps needs one, on the
  // context's own non-blocking stream (the legacy stream would also wait
  // for the work of every blocking stream)
  std::map<int, int> babies;
  {
    const int rc = plan_babies(
        c, by_n,
        [&](int n, StateView *v) {
          if (!c->cap_stream)
            TP_HIP_CHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
          return state_view(n, c->cap_stream, v);
        },
        &babies);
    if (rc != TP_OK) return rc;
  }
  int64_t extra = 0;
  for (auto &kv : by_n) {
    const int nn = kv.first;
    auto it = c->sets.find(nn);
    PowerSet probe;
    const bool fresh = it == c->sets.end() || it->second.c == 0;
    if (fresh) {
      probe.N = word_count_host(nn);
      probe.ld = probe.ld8 = (probe.N + 63) / 64 * 64;
      probe.compact = c->compact_from > 0 && nn >= c->compact_from && nn >= 2;
      probe.chain_giants = c->chain_giants_from > 0 && nn >= c->chain_giants_from;
      probe.c = babies[nn];
    }
    const PowerSet &ps = fresh ? probe : it->second;
    int top = 0;
    std::set<int> giants;
    batch_needs(kv.second, ps.c, ps.compact, ps.chain_giants, &top, &giants);
    for (int e : keys_of(top, giants, ps.c, ps.compact, ps.chain_giants))
      if (fresh || !ps.pw.count(e)) extra += ps.bytes_of(e);
  }
  return extra;
}

int tp_batch_power_trace(void *ctx, int count, const int32_t *n, const int64_t *m,
                         int32_t *gamma2_dev, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  TP_REQUIRE(count >= 0, "negative count");
  if (count == 0) return TP_OK;
  TP_REQUIRE(n && m && gamma2_dev, "NULL pointer");
  for (int j = 0; j < count; ++j) {
    TP_REQUIRE(n[j] >= 1 && n[j] <= 12, "instance %d: n = %d outside 1..12", j, n[j]);
    TP_REQUIRE(m[j] >= 3, "instance %d: m = %lld must be at least 3", j, (long long)m[j]);
    if ((int64_t)n[j] * m[j] >= 0xFFFF) {
      set_error("instance %d: n * m = %lld could reach INF", j, (long long)(n[j] * m[j]));
      return TP_EOVERFLOW;
    }
  }
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  return batch_run(c, count, n, m, gamma2_dev, stream);
}

int tp_ctx_last_work(void *ctx, double *ops, double *bytes) {
  TP_REQUIRE(ctx != nullptr && ops != nullptr && bytes != nullptr, "NULL pointer");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  for (int i = 0; i < 3; ++i) ops[i] = c->work_ops[i];
  *bytes = c->work_bytes;
  return TP_OK;
}

int tp_tune_batch(int n, int baby_steps, int fused_baby_steps) {
  TP_REQUIRE(n >= 1 && n <= 12, "n = %d outside 1..12", n);
  TP_REQUIRE(baby_steps >= 0 && baby_steps <= (1 << 16) && fused_baby_steps >= 0 &&
                 fused_baby_steps <= (1 << 16),
             "baby steps out of range");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned_baby[0][n] = baby_steps;
  g_tuned_baby[1][n] = fused_baby_steps;
  return TP_OK;
}

int tp_ctx_check(void *ctx, hipStream_t stream) {
  TP_REQUIRE(ctx != nullptr, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  return ctx_check(c, stream);
}

}  // extern "C"
